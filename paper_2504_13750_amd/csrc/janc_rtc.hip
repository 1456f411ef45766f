// janc_rtc.hip -- the chemistry kernel specialised at run time to a mechanism's structure.
//
// The generic kernel (chem_cell in janc_kernels.h) reads the species of each reaction
// from the mechanism table, so it keeps X, the Gibbs terms and the derivative row dq/dX
// in per-thread LDS columns indexed by those runtime numbers, and walks the reactions in
// a loop with wave-uniform branches. With the structure known when the source is
// compiled, those indices are constants: the same arithmetic, in the same order, runs on
// registers, and every reaction's rates can be scheduled ahead of the previous one's
// Jacobian update. Only the point-implicit cell step differs; the launch body
// (chem_body) and the solve (chem_solve) are the generic kernel's own code, compiled
// from the same headers (their texts are embedded in the library at build time).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <map>
#include <mutex>
#include <sstream>

#include "janc_rtc.h"

namespace janc {

namespace {
#include "janc_rtc_sources.inc"   // kRtcHeaderNames, kRtcHeaderTexts, kRtcHeaderCount

std::string xs(int j, int ns) { return j >= ns ? std::string("1.0") : "X[" + std::to_string(j) + "]"; }
std::string gs(int j, int ns) { return j >= ns ? std::string("0.0") : "g[" + std::to_string(j) + "]"; }
}  // namespace

std::string chem_spec_source(const DevMech& d) {
    const int ns = d.ns, nr = d.nr, nt = ns - 1;
    std::ostringstream o;
    o << "// chemistry cell step specialised to a mechanism of " << ns << " species and " << nr
      << " reactions\n#include \"janc_kernels.h\"\nnamespace janc {\n";
    o << "__device__ __forceinline__ void chem_cell_spec(CMech* m, double rho, double T, const double (&rY)["
      << nt << "], double dt, double (&w)[" << nt << "], unsigned& st) {\n";
    o << "    double X[" << ns << "];\n    double s = 0.0;\n";
    for (int j = 0; j < nt; ++j) o << "    X[" << j << "] = rY[" << j << "] * m->invM[" << j << "];\n    s += rY[" << j << "];\n";
    o << "    X[" << nt << "] = (rho - s) * m->invM[" << nt << "];\n";
    o << "    const double lnT = log(T), invT = 1.0 / T;\n";
    o << "    const double lnC = log(PATM / RU) - lnT;\n";
    o << "    double g[" << ns << "];\n#pragma unroll\n    for (int j = 0; j < " << ns << "; ++j) {\n"
         "        const bool hi = m->two_range && T >= m->tmid[j];\n        double a[7];\n#pragma unroll\n"
         "        for (int q = 0; q < 7; ++q) a[q] = hi ? m->nasa_hi[j][q] : m->nasa[j][q];\n"
         "        g[j] = a[0] * (1.0 - lnT) -\n"
         "               T * (0.5 * a[1] + T * (a[2] * (1.0 / 6.0) + T * (a[3] * (1.0 / 12.0) + T * (a[4] * 0.05)))) +\n"
         "               a[5] * invT - a[6];\n    }\n";
    o << "    double J[" << nt << "][" << nt << "];\n#pragma unroll\n    for (int k = 0; k < " << nt
      << "; ++k) {\n        w[k] = 0.0;\n#pragma unroll\n        for (int q = 0; q < " << nt
      << "; ++q) J[k][q] = 0.0;\n    }\n";
    for (int i = 0; i < nr; ++i) {
        const int* f = d.lf[i];
        const int* b = d.lb[i];
        o << "    {  // reaction " << i << "\n";
        o << "        const double lnkf = m->lnA[" << i << "] + m->b[" << i << "] * lnT - m->EaR[" << i << "] * invT;\n";
        o << "        const double kf = exp(lnkf);\n";
        if (d.rev[i]) {
            o << "        const double sg = (" << gs(b[0], ns) << " + " << gs(b[1], ns) << " + " << gs(b[2], ns) << ") - ("
              << gs(f[0], ns) << " + " << gs(f[1], ns) << " + " << gs(f[2], ns) << ");\n";
            o << "        const double kb = exp(lnkf + sg - (double)m->dnsum[" << i << "] * lnC);\n";
        } else {
            o << "        const double kb = 0.0;\n";
        }
        o << "        const double xf0 = " << xs(f[0], ns) << ", xf1 = " << xs(f[1], ns) << ", xf2 = " << xs(f[2], ns) << ";\n";
        o << "        const double xb0 = " << xs(b[0], ns) << ", xb1 = " << xs(b[1], ns) << ", xb2 = " << xs(b[2], ns) << ";\n";
        o << "        const double Rf = kf * (xf0 * xf1 * xf2), Rb = kb * (xb0 * xb1 * xb2);\n";
        if (d.has_tb[i]) {
            o << "        double ctb = 0.0;\n";
            for (int j = 0; j < ns; ++j) o << "        ctb += m->tb[" << i << "][" << j << "] * X[" << j << "];\n";
        } else {
            o << "        const double ctb = 1.0;\n";
        }
        o << "        const double net = Rf - Rb;\n        const double q = ctb * net;\n";
        for (int k = 0; k < nt; ++k) o << "        w[" << k << "] += m->Mdnu[" << i << "][" << k << "] * q;\n";
        o << "        double dq[" << ns + 1 << "];\n";
        for (int j = 0; j <= ns; ++j) {
            o << "        dq[" << j << "] = ";
            if (d.has_tb[i] && j < ns) o << "m->tb[" << i << "][" << j << "] * net;\n";
            else o << "0.0;\n";
        }
        o << "        const double cf = ctb * kf, cb = ctb * kb;\n";
        o << "        dq[" << f[0] << "] += cf * (xf1 * xf2);\n";
        o << "        dq[" << f[1] << "] += cf * (xf0 * xf2);\n";
        o << "        dq[" << f[2] << "] += cf * (xf0 * xf1);\n";
        o << "        dq[" << b[0] << "] -= cb * (xb1 * xb2);\n";
        o << "        dq[" << b[1] << "] -= cb * (xb0 * xb2);\n";
        o << "        dq[" << b[2] << "] -= cb * (xb0 * xb1);\n";
        o << "        const double dlast = dq[" << nt << "] * m->invM[" << nt << "];\n";
        o << "        double Dm[" << nt << "];\n";
        for (int mm = 0; mm < nt; ++mm) o << "        Dm[" << mm << "] = dq[" << mm << "] * m->invM[" << mm << "] - dlast;\n";
        for (int k = 0; k < nt; ++k) {
            if (d.dnu[i][k] == 0) continue;
            for (int mm = 0; mm < nt; ++mm)
                o << "        J[" << k << "][" << mm << "] += m->Mdnu[" << i << "][" << k << "] * Dm[" << mm << "];\n";
        }
        o << "    }\n";
    }
    o << "    chem_solve<" << ns << ">(J, w, dt, st);\n}\n}  // namespace janc\n";
    o << "extern \"C\" __global__ __launch_bounds__(janc::WG, 2) void " << CHEM_SPEC_KERNEL
      << "(janc::StageArgs a) {\n    __shared__ double scratch[16];\n    janc::chem_body<" << ns
      << ">(a, scratch, [&](janc::CMech* m, double rho, double T, const double (&rY)[" << nt
      << "], double dt, double (&dY)[" << nt << "], unsigned& st) {\n"
         "        janc::chem_cell_spec(m, rho, T, rY, dt, dY, st);\n    });\n}\n";
    return o.str();
}

bool chem_spec_code(const std::string& src, std::vector<char>* code, std::string* log) {
    static std::mutex mu;
    static std::map<std::string, std::vector<char>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(src);
    if (it != cache.end()) {
        *code = it->second;
        return true;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "janc_chem_spec.hip", kRtcHeaderCount, kRtcHeaderTexts,
                            kRtcHeaderNames) != HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    // the library's own build flags (fused multiply-add only within an expression, no
    // packed FP32 instructions)
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=on",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-Wno-unused-value", "-Wno-unused-result"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t n = 0;
    if (r != HIPRTC_SUCCESS) {
        hiprtcGetProgramLogSize(prog, &n);
        log->assign(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &(*log)[0]);
        hiprtcDestroyProgram(&prog);
        return false;
    }
    hiprtcGetCodeSize(prog, &n);
    code->assign(n, 0);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    cache[src] = *code;
    return true;
}

}  // namespace janc
