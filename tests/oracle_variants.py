"""Run an oracle computation in a child process with another build of the oracle.

The oracle has one build per process (loaded once through ctypes). The "fma" build
(the same source compiled with fused multiply-add contraction) serves only to measure
the oracle's own round-off floor: how far a result moves when every a*b+c is rounded
once instead of twice. `in_variant("fma", "module:function", kwargs)` imports the
function in a child process that loads that build and returns its JSON-serializable
result.
"""

import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def in_variant(variant, target, kwargs):
    mod, fn = target.split(":")
    code = ("import json, sys, importlib; "
            f"sys.path[:0] = [{ROOT!r}, {HERE!r}]; "
            f"f = getattr(importlib.import_module({mod!r}), {fn!r}); "
            "print('__RESULT__' + json.dumps(f(**json.loads(sys.argv[1]))))")
    env = dict(os.environ, JANC_ORACLE_VARIANT=variant)
    r = subprocess.run([sys.executable, "-c", code, json.dumps(kwargs)], env=env,
                       capture_output=True, text=True, check=True)
    line = [x for x in r.stdout.splitlines() if x.startswith("__RESULT__")][-1]
    return json.loads(line[len("__RESULT__"):])
