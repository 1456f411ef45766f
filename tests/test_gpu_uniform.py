"""GPU parity on uniform grids: the HIP path (through the C ABI) against the CPU
oracle on the same seeded inputs.

Bar: max relative error per conserved field <= 1e-10 (field-max normalization),
temperatures likewise; time steps to 1e-12. Sizes span several tiles and
ragged tails; the full 1024 x 128 detonation tube runs in the launch
configuration the benchmark times.
"""

import numpy as np
import pytest

import oracle
from cases import (sod_case, detonation_tube_case, Case, MODEL_CPG, MODEL_ONESTEP, BC_PERIODIC,
                   BC_ZEROGRAD, BC_SLIPWALL, BC_DIRICHLET, MODEL_DETAILED, synthetic_mechanism)
from cases.amr import detailed_front_case
from gpu_util import run_uniform, rel_err, context_for, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _compare(case, nsteps, tol=TOL, **kw):
    Ug, Tg, tg, dg = run_uniform(case, nsteps, **kw)
    Uo, To = oracle.case_state(case)
    okw = {k: v for k, v in kw.items() if k in ("dt_fixed", "t_end", "cfl")}
    okw["strang"] = kw.get("split", 0) == 1
    okw["full_jacobian"] = kw.get("jac", 0) == 1
    Uo, To, to, do, _ = oracle.step(case, Uo, To, nsteps, **okw)
    e = rel_err(Ug, Uo)
    eT = rel_err(Tg[None], To[None])[0]
    print(f"  {case.name}: per-field rel err {np.array2string(e, precision=2)}, T {eT:.2e}, "
          f"t gpu {tg:.12e} oracle {to:.12e}", flush=True)
    assert np.all(e <= tol), e
    assert eT <= tol
    assert tg == pytest.approx(to, rel=1e-12)
    assert np.allclose(dg, do, rtol=1e-12, atol=0.0)
    return Ug, Uo


@pytest.mark.parametrize("model", ["cpg", "onestep", "detailed"])
def test_init_state_parity(model):
    torch, dev = torch_dev()
    if model == "cpg":
        c = sod_case(nx=64)
    elif model == "onestep":
        c = detonation_tube_case(nx=40, ny=8, seed=3)
    else:
        c = detailed_front_case(nx=24, ny=8)
    ctx = context_for(c)
    import paper_2504_13750_amd as janc
    U, T = ctx.init_state(janc.physics_of(c), torch.tensor(c.W, dtype=torch.float64, device=dev))
    Uo, To = oracle.case_state(c)
    assert np.all(rel_err(U.cpu().numpy(), Uo) <= 1e-14)
    assert np.all(rel_err(T.cpu().numpy()[None], To[None]) <= 1e-14)
    ctx.close()


def test_sod_full_run():
    """Sod problem: 400 cells, CFL 0.5 to t = 0.2 (last step clipped, later steps no-ops)."""
    c = sod_case()
    _compare(c, 400)


def test_detonation_ragged_tiles():
    # 100 x 20: neither 16 nor 32 divides the grid, so tiles have ragged tails
    _compare(detonation_tube_case(nx=100, ny=20, seed=21), 120)


def test_detonation_many_steps_small():
    _compare(detonation_tube_case(nx=128, ny=32, seed=22), 400)


@pytest.mark.timeout(900)
def test_detonation_tube_1024x128_to_1000_steps():
    """The full 1024 x 128 tube over its stated 1000 steps, compared every 100 steps. The
    front is unstable, so round-off grows with N: each field is held to max(1e-10, 2 x the
    oracle's own floor at N): the larger change of the oracle's result under a one-ulp
    density change or under fused multiply-add contraction (tests/golden/
    tube_1024x128_floor.json, written by tests/golden/make_floors.py)."""
    import paper_2504_13750_amd as janc
    from test_oracle_floors import tube_floor_golden
    floor = tube_floor_golden()
    c = detonation_tube_case()
    torch, dev = torch_dev()
    ctx = context_for(c)
    phys = janc.physics_of(c)
    U, T = ctx.init_state(phys, torch.tensor(c.W, dtype=torch.float64, device=dev))
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    Uo, To = oracle.case_state(c)
    to, n = 0.0, 0
    for N in sorted(floor):
        print(f"[gpu] janc_step {c.name} 1024x128 steps {n}..{N}", flush=True)
        ctx.step(janc.grid_of(c), phys, janc.time_of(c), U, T, N - n, t)
        ctx.sync_status()
        Uo, To, to, _, _ = oracle.step(c, Uo, To, N - n, t=to)
        n = N
        e = rel_err(U.cpu().numpy(), Uo)
        bar = np.maximum(TOL, 2.0 * floor[N])
        print(f"  N={N}: per-field rel err {np.array2string(e, precision=2)}, floor "
              f"{np.array2string(floor[N], precision=2)}", flush=True)
        assert np.all(e <= bar), (N, e, bar)
        assert t.item() == pytest.approx(to, rel=1e-12)
    ctx.close()


@pytest.mark.parametrize("shape", [(3, 3), (5, 1), (3, 1), (17, 9), (256, 1), (700, 1)])
def test_small_and_one_dimensional_grids(shape):
    nx, ny = shape
    rng = np.random.default_rng(nx * 31 + ny)
    W = np.zeros((5, ny, nx))
    W[0] = 1.0 + 0.2 * rng.uniform(size=(ny, nx))
    W[1] = 0.3 * rng.normal(size=(ny, nx))
    W[2] = 0.0 if ny == 1 else 0.3 * rng.normal(size=(ny, nx))
    W[3] = 1.0 + rng.uniform(size=(ny, nx))
    W[4] = rng.uniform(size=(ny, nx))
    c = Case(name=f"rand{nx}x{ny}", model=MODEL_ONESTEP, nx=nx, ny=ny, dx=0.05, dy=0.07,
             bc=[BC_PERIODIC, BC_PERIODIC, BC_SLIPWALL, BC_SLIPWALL], W=W, gamma=1.25, R=1.0,
             Q=3.0, Ea=4.0, k=2.0, cfl=0.45)
    _compare(c, 30)


@pytest.mark.parametrize("bc", [(BC_ZEROGRAD, BC_ZEROGRAD, BC_ZEROGRAD, BC_ZEROGRAD),
                                (BC_SLIPWALL, BC_DIRICHLET, BC_PERIODIC, BC_PERIODIC),
                                (BC_DIRICHLET, BC_SLIPWALL, BC_DIRICHLET, BC_ZEROGRAD)])
def test_boundary_kinds(bc):
    c = detonation_tube_case(nx=48, ny=24, seed=5)
    c.bc = list(bc)
    st = np.array([1.1, 0.2, -0.1, 1.3, 0.9])
    c.bc_prim = [st if b == BC_DIRICHLET else None for b in bc]
    _compare(c, 40)


def test_cpg_two_dimensional_fixed_dt():
    rng = np.random.default_rng(12)
    nx, ny = 64, 48
    W = np.zeros((4, ny, nx))
    W[0] = 1.0 + 0.5 * (rng.uniform(size=(ny, nx)) > 0.5)
    W[1] = 0.1 * rng.normal(size=(ny, nx))
    W[2] = 0.1 * rng.normal(size=(ny, nx))
    W[3] = 1.0 + (rng.uniform(size=(ny, nx)) > 0.7)
    c = Case(name="cpg2d", model=MODEL_CPG, nx=nx, ny=ny, dx=0.01, dy=0.01,
             bc=[BC_SLIPWALL, BC_ZEROGRAD, BC_PERIODIC, BC_PERIODIC], W=W, gamma=1.4, R=287.0)
    _compare(c, 50, dt_fixed=1e-3)


def test_detailed_front_uniform():
    """9-species front (NASA-7 Newton + point-implicit chemistry) on a uniform grid."""
    c = detailed_front_case(nx=48, ny=40)
    _compare(c, 4)


def test_detailed_front_two_range_thermo():
    """The same front with two-range NASA-7 data switching at 1800 K, inside the front's
    1200-2500 K span, so Newton, the Gibbs terms and the initial energy use both sets."""
    from cases import synthetic_mechanism, two_range_mechanism
    c = detailed_front_case(nx=48, ny=40, mech=two_range_mechanism(synthetic_mechanism()))
    _compare(c, 4)


def test_species_dependent_t_mid_rejected():
    import copy
    import paper_2504_13750_amd as janc
    from cases import synthetic_mechanism, two_range_mechanism
    m = copy.deepcopy(two_range_mechanism(synthetic_mechanism()))
    m.t_mid[2] = 1500.0
    with pytest.raises(janc.JancError) as ei:
        janc.Context(janc.DETAILED, m)
    assert ei.value.code == -1


def test_zero_steps_only_resolves_temperature():
    c = detailed_front_case(nx=32, ny=16)
    Ug, Tg, tg, _ = run_uniform(c, 0)
    Uo, To = oracle.case_state(c)
    assert np.array_equal(Ug, Uo) or np.all(rel_err(Ug, Uo) <= 1e-15)
    assert tg == 0.0


def test_status_flag_on_negative_density():
    """A state with negative pressure is reported through the sticky status word."""
    import paper_2504_13750_amd as janc
    c = detonation_tube_case(nx=32, ny=8, seed=1)
    c.W[3, 4, 10] = -5.0           # negative pressure in one cell
    with pytest.raises(janc.JancError) as ei:
        run_uniform(c, 1)
    assert ei.value.code == -6


def test_status_flag_on_non_finite_state():
    """A NaN density is reported as JANC_ENONFINITE through the sticky status word, and the
    word is cleared once read."""
    import paper_2504_13750_amd as janc
    c = detonation_tube_case(nx=32, ny=8, seed=1)
    c.W[0, 4, 10] = float("nan")
    with pytest.raises(janc.JancError) as ei:
        run_uniform(c, 1)
    assert ei.value.code == -4
    ok = detonation_tube_case(nx=32, ny=8, seed=1)
    run_uniform(ok, 1)        # a fresh context reports no stale status


def test_detailed_front_strang_splitting():
    c = detailed_front_case(nx=48, ny=40)
    _compare(c, 4, split=1)


def test_strang_rejected_without_chemistry():
    import paper_2504_13750_amd as janc
    c = detonation_tube_case(nx=16, ny=8, seed=3)
    with pytest.raises(janc.JancError) as ei:
        run_uniform(c, 1, split=1)
    assert ei.value.code == -1


def test_detailed_front_full_jacobian():
    c = detailed_front_case(nx=48, ny=40)
    _compare(c, 4, jac=1)


def test_detailed_front_full_jacobian_two_range_strang():
    from cases import synthetic_mechanism, two_range_mechanism
    c = detailed_front_case(nx=48, ny=40, mech=two_range_mechanism(synthetic_mechanism()))
    _compare(c, 4, jac=1, split=1)


def test_chemkin_loaded_mechanism_drives_the_library():
    """A mechanism written to chemkin text and read back (two NASA-7 ranges) runs the
    9-species front like the oracle does with the same loaded mechanism."""
    from paper_2504_13750_amd import chemkin
    from cases import synthetic_mechanism, two_range_mechanism
    m0 = two_range_mechanism(synthetic_mechanism())
    m = chemkin.parse(chemkin.write(m0, atomic_weights={"A": 2.0, "B": 16.0, "C": 14.0}),
                      complement="C2")
    c = detailed_front_case(nx=48, ny=40, mech=m)
    _compare(c, 4)


def test_full_jacobian_rejected_without_chemistry():
    import paper_2504_13750_amd as janc
    c = detonation_tube_case(nx=16, ny=8, seed=3)
    with pytest.raises(janc.JancError) as ei:
        run_uniform(c, 1, jac=1)
    assert ei.value.code == -1


@pytest.mark.parametrize("start", ["atoms-600K", "fresh-1500K"])
def test_adiabatic_reactor_reaches_gibbs_equilibrium(start):
    """An 8 x 8 periodic grid in one 0-D state with the complete-channel mechanism (30
    reactions), 200 steps each of 1e-10, 1e-9, 1e-8 and 1e-7 s: the GPU matches the oracle
    and its temperature is the independent Gibbs equilibrium temperature of the mixture.
    Bar per field: max(1e-10, 2 x the oracle's floor), the floor measured here as the
    oracle's own change under a +-1e-15 relative change of the initial species densities
    (rounding level from the atoms; above 1e-10 from the fresh mixture, whose relaxation
    is ill-conditioned)."""
    import refsol
    from cases.mechanism import complete_mechanism
    from test_oracle_floors import reactor_case, reactor_floor, REACTOR_DTS
    mech = complete_mechanism()
    c = reactor_case(mech, start, n=8)
    import paper_2504_13750_amd as janc
    print(f"[gpu] janc_step {c.name} 8x8, 4 x 200 steps", flush=True)
    torch, dev = torch_dev()
    ctx = context_for(c)
    phys = janc.physics_of(c)
    U, T = ctx.init_state(phys, torch.tensor(c.W, dtype=torch.float64, device=dev))
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    for dt in REACTOR_DTS:
        ctx.step(janc.grid_of(c), phys, janc.time_of(c, dt_fixed=dt), U, T, 200, t)
    ctx.sync_status()
    Ug, Tg = U.cpu().numpy(), T.cpu().numpy()
    ctx.close()
    Uo, To = oracle.case_state(c)
    rho, e = Uo[0, 0, 0], Uo[3, 0, 0] / Uo[0, 0, 0]
    X0 = np.r_[Uo[4:, 0, 0], rho - Uo[4:, 0, 0].sum()] / mech.M
    Teq, Xeq = refsol.equilibrium_T(mech, rho, e, mech.comp.T.astype(float) @ X0)
    for dt in REACTOR_DTS:
        Uo, To, _, _, _ = oracle.step(c, Uo, To, 200, dt_fixed=dt)
    err = rel_err(Ug, Uo)
    bar = np.maximum(TOL, 2.0 * reactor_floor(oracle, start))
    print(f"  reactor {start}: GPU T {Tg[0, 0]:.10f}, Gibbs {Teq:.10f}, per-field rel err "
          f"{np.array2string(err, precision=2)}, bar {np.array2string(bar, precision=2)}",
          flush=True)
    assert np.all(err <= bar)
    assert Tg[0, 0] == pytest.approx(Teq, rel=1e-9)
    X = np.r_[Ug[4:, 0, 0], rho - Ug[4:, 0, 0].sum()] / mech.M
    assert np.max(np.abs(X - Xeq)) <= 1e-7 * X.sum()
