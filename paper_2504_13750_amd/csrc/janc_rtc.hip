// janc_rtc.hip -- the chemistry kernels specialised at run time to a mechanism's structure:
// the point-implicit step of the forward path and its reverse in the discrete adjoint.
//
// The generic kernel (chem_cell in janc_kernels.h) reads the species of each reaction
// from the mechanism table, so it keeps X, the Gibbs terms and the derivative row dq/dX
// in per-thread LDS columns indexed by those runtime numbers, and walks the reactions in
// a loop with wave-uniform branches. With the structure known when the source is
// compiled, those indices are constants: the same arithmetic, in the same order, runs on
// registers, and every reaction's rates can be scheduled ahead of the previous one's
// Jacobian update. The mechanism's numbers become exact hexadecimal literals (no scalar
// loads and waits for them), except the NASA-7 coefficients, whose products with the
// polynomial's constant factors would otherwise be folded at compile time and round
// differently from the generic kernel. Only the point-implicit cell step differs; the launch body
// (chem_body) and the solve (chem_solve) are the generic kernel's own code, compiled
// from the same headers (their texts are embedded in the library at build time).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <sstream>

#include "janc_rtc.h"

namespace janc {

namespace {
#include "janc_rtc_sources.inc"   // kRtcHeaderNames, kRtcHeaderTexts, kRtcHeaderCount

std::string xs(int j, int ns) { return j >= ns ? std::string("1.0") : "X[" + std::to_string(j) + "]"; }
std::string gs(int j, int ns) { return j >= ns ? std::string("0.0") : "g[" + std::to_string(j) + "]"; }
// A number of the mechanism as an exact hexadecimal literal.
std::string lit(double v) {
    char buf[48];
    std::snprintf(buf, sizeof buf, "(%a)", v);
    return buf;
}
}  // namespace

std::string chem_spec_source(const DevMech& d) {
    const int ns = d.ns, nr = d.nr, nt = ns - 1;
    std::ostringstream o;
    o << "// chemistry cell step specialised to a mechanism of " << ns << " species and " << nr
      << " reactions\n#include \"janc_kernels.h\"\nnamespace janc {\n";
    o << "__device__ __forceinline__ void chem_cell_spec(CMech* m, double rho, double T, const double (&rY)["
      << nt << "], double dt, double (&w)[" << nt << "], unsigned& st) {\n";
    o << "    double X[" << ns << "];\n    double s = 0.0;\n";
    for (int j = 0; j < nt; ++j) o << "    X[" << j << "] = rY[" << j << "] * " << lit(d.invM[j]) << ";\n    s += rY[" << j << "];\n";
    o << "    X[" << nt << "] = (rho - s) * " << lit(d.invM[nt]) << ";\n";
    o << "    const double lnT = log(T), invT = 1.0 / T;\n";
    o << "    const double lnC = log(PATM / RU) - lnT;\n";
    // the NASA-7 coefficients stay table reads: as literals, their products with the
    // polynomial's constant factors would be folded at compile time (rounded once, where
    // the generic kernel fuses them into the next multiply-add)
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
        o << "        const double lnkf = " << lit(d.lnA[i]) << " + " << lit(d.b[i]) << " * lnT - " << lit(d.EaR[i]) << " * invT;\n";
        o << "        const double kf = exp(lnkf);\n";
        if (d.rev[i]) {
            o << "        const double sg = (" << gs(b[0], ns) << " + " << gs(b[1], ns) << " + " << gs(b[2], ns) << ") - ("
              << gs(f[0], ns) << " + " << gs(f[1], ns) << " + " << gs(f[2], ns) << ");\n";
            o << "        const double kb = exp(lnkf + sg - " << lit((double)d.dnsum[i]) << " * lnC);\n";
        } else {
            o << "        const double kb = 0.0;\n";
        }
        o << "        const double xf0 = " << xs(f[0], ns) << ", xf1 = " << xs(f[1], ns) << ", xf2 = " << xs(f[2], ns) << ";\n";
        o << "        const double xb0 = " << xs(b[0], ns) << ", xb1 = " << xs(b[1], ns) << ", xb2 = " << xs(b[2], ns) << ";\n";
        o << "        const double Rf = kf * (xf0 * xf1 * xf2), Rb = kb * (xb0 * xb1 * xb2);\n";
        if (d.has_tb[i]) {
            o << "        double ctb = 0.0;\n";
            for (int j = 0; j < ns; ++j) o << "        ctb += " << lit(d.tb[i][j]) << " * X[" << j << "];\n";
        } else {
            o << "        const double ctb = 1.0;\n";
        }
        o << "        const double net = Rf - Rb;\n        const double q = ctb * net;\n";
        for (int k = 0; k < nt; ++k) o << "        w[" << k << "] += " << lit(d.Mdnu[i][k]) << " * q;\n";
        o << "        double dq[" << ns + 1 << "];\n";
        for (int j = 0; j <= ns; ++j) {
            o << "        dq[" << j << "] = ";
            if (d.has_tb[i] && j < ns) o << "" << lit(d.tb[i][j]) << " * net;\n";
            else o << "0.0;\n";
        }
        o << "        const double cf = ctb * kf, cb = ctb * kb;\n";
        o << "        dq[" << f[0] << "] += cf * (xf1 * xf2);\n";
        o << "        dq[" << f[1] << "] += cf * (xf0 * xf2);\n";
        o << "        dq[" << f[2] << "] += cf * (xf0 * xf1);\n";
        o << "        dq[" << b[0] << "] -= cb * (xb1 * xb2);\n";
        o << "        dq[" << b[1] << "] -= cb * (xb0 * xb2);\n";
        o << "        dq[" << b[2] << "] -= cb * (xb0 * xb1);\n";
        o << "        const double dlast = dq[" << nt << "] * " << lit(d.invM[nt]) << ";\n";
        o << "        double Dm[" << nt << "];\n";
        for (int mm = 0; mm < nt; ++mm) o << "        Dm[" << mm << "] = dq[" << mm << "] * " << lit(d.invM[mm]) << " - dlast;\n";
        for (int k = 0; k < nt; ++k) {
            if (d.dnu[i][k] == 0) continue;
            for (int mm = 0; mm < nt; ++mm)
                o << "        J[" << k << "][" << mm << "] += " << lit(d.Mdnu[i][k]) << " * Dm[" << mm << "];\n";
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

std::string adj_chem_spec_source(const DevMech& d) {
    const int ns = d.ns, nr = d.nr, nt = ns - 1;
    const std::string NS = std::to_string(ns), NT = std::to_string(nt);
    std::ostringstream o;
    o << "// reversed chemistry cell step specialised to a mechanism of " << ns << " species and " << nr
      << " reactions\n#include \"janc_adjoint.h\"\nnamespace janc {\nstruct AdjReactionsSpec {\n";
    // the forward rates, S and J (AdjReactions::rates with the structure compiled in)
    o << "    __device__ __forceinline__ void rates(CMech* m, const double (&X)[" << ns + 1
      << "], double lnT, double invT, double lnC, const double (&gts)[" << ns + 1 << "], double (&S)[" << NT
      << "], double (&J)[" << NT << "][" << NT << "]) const {\n";
    for (int i = 0; i < nr; ++i) {
        const int* f = d.lf[i];
        const int* b = d.lb[i];
        const std::string I = std::to_string(i);
        o << "        {  // reaction " << i << "\n";
        o << "            const double lnkf = " << lit(d.lnA[i]) << " + " << lit(d.b[i]) << " * lnT - " << lit(d.EaR[i]) << " * invT;\n";
        o << "            const double kf = exp(lnkf);\n            double kb = 0.0;\n";
        if (d.rev[i]) {
            o << "            {\n                double sg = 0.0;\n";
            for (int q = 0; q < MAXLIST; ++q)
                o << "                sg += gts[" << b[q] << "] - gts[" << f[q] << "];\n";
            o << "                kb = exp(lnkf + sg - " << lit((double)d.dnsum[i]) << " * lnC);\n            }\n";
        }
        o << "            const double Rf = kf * (X[" << f[0] << "] * X[" << f[1] << "] * X[" << f[2]
          << "]), Rb = kb * (X[" << b[0] << "] * X[" << b[1] << "] * X[" << b[2] << "]);\n";
        if (d.has_tb[i]) {
            o << "            double ctb = 0.0;\n";
            for (int j = 0; j < ns; ++j) o << "            ctb += " << lit(d.tb[i][j]) << " * X[" << j << "];\n";
        } else {
            o << "            const double ctb = 1.0;\n";
        }
        o << "            const double q = ctb * (Rf - Rb);\n";
        for (int k = 0; k < nt; ++k) o << "            S[" << k << "] += " << lit(d.Mdnu[i][k]) << " * q;\n";
        o << "            double dq[" << ns + 1 << "];\n";
        for (int j = 0; j <= ns; ++j) {
            if (d.has_tb[i] && j < ns) o << "            dq[" << j << "] = " << lit(d.tb[i][j]) << " * (Rf - Rb);\n";
            else o << "            dq[" << j << "] = 0.0;\n";
        }
        o << "            dq[" << f[0] << "] += ctb * kf * (X[" << f[1] << "] * X[" << f[2] << "]);\n";
        o << "            dq[" << f[1] << "] += ctb * kf * (X[" << f[0] << "] * X[" << f[2] << "]);\n";
        o << "            dq[" << f[2] << "] += ctb * kf * (X[" << f[0] << "] * X[" << f[1] << "]);\n";
        o << "            dq[" << b[0] << "] -= ctb * kb * (X[" << b[1] << "] * X[" << b[2] << "]);\n";
        o << "            dq[" << b[1] << "] -= ctb * kb * (X[" << b[0] << "] * X[" << b[2] << "]);\n";
        o << "            dq[" << b[2] << "] -= ctb * kb * (X[" << b[0] << "] * X[" << b[1] << "]);\n";
        o << "            const double dl = dq[" << nt << "] * " << lit(d.invM[nt]) << ";\n";
        for (int k = 0; k < nt; ++k) {
            if (d.dnu[i][k] == 0) continue;
            for (int q2 = 0; q2 < nt; ++q2)
                o << "            J[" << k << "][" << q2 << "] += " << lit(d.Mdnu[i][k]) << " * (dq[" << q2
                  << "] * " << lit(d.invM[q2]) << " - dl);\n";
        }
        o << "        }\n";
    }
    o << "    }\n";
    // the reverse sweep (AdjReactions::sweep with the structure compiled in)
    o << "    __device__ __forceinline__ void sweep(CMech* m, const double (&X)[" << ns + 1
      << "], const double (&dX)[" << ns + 1 << "], const double (&mu)[" << NT
      << "], double lnT, double invT, double lnC, const double (&gts)[" << ns + 1 << "], const double (&hm1)["
      << ns + 1 << "], double (&G)[" << ns + 1 << "], double& GT) const {\n";
    for (int i = 0; i < nr; ++i) {
        const int* f = d.lf[i];
        const int* b = d.lb[i];
        const std::string I = std::to_string(i);
        o << "        {  // reaction " << i << "\n            double ci = 0.0;\n";
        for (int k = 0; k < nt; ++k) o << "            ci += mu[" << k << "] * " << lit(d.Mdnu[i][k]) << ";\n";
        o << "            if (ci != 0.0) {\n";
        o << "                const double lnkf = " << lit(d.lnA[i]) << " + " << lit(d.b[i]) << " * lnT - " << lit(d.EaR[i]) << " * invT;\n";
        o << "                const double kf = exp(lnkf);\n                double kb = 0.0, dlb = 0.0;\n";
        o << "                const double dlf = (" << lit(d.b[i]) << " + " << lit(d.EaR[i]) << " * invT) * invT;\n";
        if (d.rev[i]) {
            o << "                {\n                    double sg = 0.0, sh = 0.0;\n";
            for (int q = 0; q < MAXLIST; ++q) {
                o << "                    sg += gts[" << b[q] << "] - gts[" << f[q] << "];\n";
                o << "                    sh += hm1[" << b[q] << "] - hm1[" << f[q] << "];\n";
            }
            o << "                    kb = exp(lnkf + sg - " << lit((double)d.dnsum[i]) << " * lnC);\n";
            o << "                    dlb = dlf - sh * invT;\n                }\n";
        }
        // R = k x0 x1 x2, dR/dx_s, dR . dX and its gradient, for the reactants (F) and,
        // if reversible, the products (B); zero otherwise
        auto prod = [&](const char* P, const int* sl, const char* kk) {
            o << "                const double " << P << "x0 = X[" << sl[0] << "], " << P << "x1 = X[" << sl[1] << "], "
              << P << "x2 = X[" << sl[2] << "];\n";
            o << "                const double " << P << "e0 = dX[" << sl[0] << "], " << P << "e1 = dX[" << sl[1] << "], "
              << P << "e2 = dX[" << sl[2] << "];\n";
            o << "                const double R" << P << " = " << kk << " * (" << P << "x0 * " << P << "x1 * " << P << "x2);\n";
            o << "                const double dR" << P << "0 = " << kk << " * (" << P << "x1 * " << P << "x2), dR" << P
              << "1 = " << kk << " * (" << P << "x0 * " << P << "x2), dR" << P << "2 = " << kk << " * (" << P << "x0 * "
              << P << "x1);\n";
            o << "                const double dR" << P << "d = dR" << P << "0 * " << P << "e0 + dR" << P << "1 * " << P
              << "e1 + dR" << P << "2 * " << P << "e2;\n";
            o << "                const double ddR" << P << "0 = " << kk << " * (" << P << "e1 * " << P << "x2 + " << P
              << "x1 * " << P << "e2), ddR" << P << "1 = " << kk << " * (" << P << "e0 * " << P << "x2 + " << P << "x0 * "
              << P << "e2), ddR" << P << "2 = " << kk << " * (" << P << "e0 * " << P << "x1 + " << P << "x0 * " << P
              << "e1);\n";
        };
        prod("F", f, "kf");
        if (d.rev[i]) {
            prod("B", b, "kb");
        } else {
            o << "                const double RB = 0.0, dRB0 = 0.0, dRB1 = 0.0, dRB2 = 0.0, dRBd = 0.0, ddRB0 = 0.0, "
                 "ddRB1 = 0.0, ddRB2 = 0.0;\n";
        }
        if (d.has_tb[i]) {
            o << "                double ctb = 0.0, dctb = 0.0;\n";
            for (int j = 0; j < ns; ++j) {
                o << "                ctb += " << lit(d.tb[i][j]) << " * X[" << j << "];\n";
                o << "                dctb += " << lit(d.tb[i][j]) << " * dX[" << j << "];\n";
            }
        } else {
            o << "                const double ctb = 1.0, dctb = 0.0;\n";
        }
        o << "                const double net = RF - RB, dnet = dRFd - dRBd;\n";
        if (d.has_tb[i])
            for (int j = 0; j < ns; ++j)
                o << "                G[" << j << "] += ci * " << lit(d.tb[i][j]) << " * (net + dnet);\n";
        for (int q = 0; q < 3; ++q) {
            o << "                G[" << f[q] << "] += ci * ((ctb + dctb) * dRF" << q << " + ctb * ddRF" << q << ");\n";
            o << "                G[" << b[q] << "] -= ci * ((ctb + dctb) * dRB" << q << " + ctb * ddRB" << q << ");\n";
        }
        o << "                GT += ci * ((ctb + dctb) * (RF * dlf - RB * dlb) + ctb * (dRFd * dlf - dRBd * dlb));\n";
        o << "            }\n        }\n";
    }
    o << "    }\n};\n}  // namespace janc\n";
    o << "extern \"C\" __global__ __launch_bounds__(janc::AWG) void " << ADJ_CHEM_SPEC_KERNEL
      << "(janc::AdjChemArgs A) {\n    janc::adj_chem_cell<" << ns << ">(A, janc::AdjReactionsSpec{});\n}\n";
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
