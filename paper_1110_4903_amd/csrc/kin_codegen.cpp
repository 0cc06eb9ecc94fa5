// kin_codegen.cpp -- mechanism validation, preprocessing and the lane-layout code generator.
//
// The lane layout keeps one cell's whole Newton system in the registers of one lane.  A
// register file can only be addressed by compile-time indices, so the mechanism's structure
// (which species take part in which reaction, with which coefficients) is compiled into the
// kernel: kin_mech_upload generates straight-line code for the rates, the production terms
// and the analytic Jacobian of that mechanism and compiles it with hipRTC for gfx950.
#include <hip/hiprtc.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <sstream>

#include "kin_internal.h"

namespace kin {

static const char kLaneTemplate[] =
#include "kin_lane_template.inc"
    ;

bool MechHost::single_range(int s) const
{
    for (int k = 0; k < 7; ++k)
        if (nasa[14 * s + k] != nasa[14 * s + 7 + k]) return false;
    return true;
}

static bool finite(double v) { return std::isfinite(v); }

kin_status mech_from_desc(const kin_mech_desc *d, MechHost &m, std::string &msg)
{
    auto fail = [&](const std::string &s) { msg = "mechanism: " + s; return KIN_EINVAL; };
    if (!d) return fail("NULL descriptor");
    if (d->ns < 1 || d->ns > kNsMax) return fail("ns must be in 1..255");
    if (d->ne < 1 || d->nr < 1 || d->ntb < 0) return fail("ne >= 1, nr >= 1, ntb >= 0 required");
    if (!d->M || !d->elem || !d->nasa || !d->T_mid || !d->reac_idx || !d->reac_nu ||
        !d->prod_idx || !d->prod_nu || !d->A || !d->b || !d->Ta || !d->reversible || !d->tb ||
        (d->ntb > 0 && !d->eff))
        return fail("NULL array");
    m = MechHost();
    m.ns = d->ns; m.ne = d->ne; m.nr = d->nr; m.ntb = d->ntb;
    m.M.assign(d->M, d->M + m.ns);
    m.nasa.assign(d->nasa, d->nasa + 14 * m.ns);
    m.Tmid.assign(d->T_mid, d->T_mid + m.ns);
    m.elem.assign(d->elem, d->elem + m.ns * m.ne);
    if (m.ntb) m.eff.assign(d->eff, d->eff + (size_t)m.ntb * m.ns);
    for (int s = 0; s < m.ns; ++s) {
        if (!(m.M[s] > 0) || !finite(m.M[s])) return fail("molar mass must be positive");
        if (!(m.Tmid[s] > 0) || !finite(m.Tmid[s])) return fail("T_mid must be positive");
        for (int k = 0; k < 14; ++k) if (!finite(m.nasa[14 * s + k])) return fail("non-finite NASA coefficient");
        for (int e = 0; e < m.ne; ++e) if (m.elem[s * m.ne + e] < 0) return fail("negative element count");
        // c_v = R (cp/R - 1) must stay positive over the admissible temperature range
        for (double T = 200.0; T <= 6000.0; T += 10.0) {
            const double *a = &m.nasa[14 * s + (T < m.Tmid[s] ? 0 : 7)];
            double cp = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
            if (!(cp > 1.0)) return fail("cp/R must exceed 1 on [200, 6000] K (species " + std::to_string(s) + ")");
        }
    }
    for (double v : m.eff) if (!(v >= 0) || !finite(v)) return fail("efficiencies must be finite and >= 0");
    m.rx.resize(m.nr);
    for (int r = 0; r < m.nr; ++r) {
        Rxn &x = m.rx[r];
        std::memset(&x, 0, sizeof(x));
        x.A = d->A[r]; x.b = d->b[r]; x.Ta = d->Ta[r];
        if (!(x.A > 0) || !finite(x.A) || !finite(x.b) || !finite(x.Ta)) return fail("bad Arrhenius parameters in reaction " + std::to_string(r));
        x.lnA = std::log(x.A);
        x.rev = d->reversible[r] ? 1 : 0;
        x.tb = d->tb[r];
        if (x.tb < -1 || x.tb >= m.ntb) return fail("third-body row out of range");
        std::vector<int> bal(m.ne, 0);
        for (int side = 0; side < 2; ++side) {
            const int32_t *idx = side ? d->prod_idx + 3 * r : d->reac_idx + 3 * r;
            const int32_t *nu = side ? d->prod_nu + 3 * r : d->reac_nu + 3 * r;
            int *msp = side ? x.prod_sp : x.reac_sp;
            int *mnu = side ? x.prod_nu : x.reac_nu;
            int &cnt = side ? x.nprod : x.nreac;
            for (int j = 0; j < 3; ++j) {
                if (idx[j] < 0) continue;
                if (idx[j] >= m.ns) return fail("species index out of range");
                if (nu[j] < 1 || nu[j] > 3) return fail("stoichiometric coefficients must be 1..3");
                int k = 0;
                while (k < cnt && msp[k] != idx[j]) ++k;
                if (k == cnt) { msp[cnt] = idx[j]; mnu[cnt] = 0; ++cnt; }
                mnu[k] += nu[j];
                for (int e = 0; e < m.ne; ++e) bal[e] += (side ? 1 : -1) * nu[j] * m.elem[idx[j] * m.ne + e];
            }
        }
        if (x.nreac == 0 || x.nprod == 0) return fail("reaction without reactants or products");
        for (int e = 0; e < m.ne; ++e) if (bal[e]) return fail("reaction " + std::to_string(r) + " is not element-balanced");
        for (int k = 0; k < x.nreac; ++k) if (x.reac_nu[k] > 3) return fail("total coefficient above 3");
        for (int k = 0; k < x.nprod; ++k) if (x.prod_nu[k] > 3) return fail("total coefficient above 3");
        x.dnu = 0;
        for (int k = 0; k < x.nprod; ++k) x.dnu += x.prod_nu[k];
        for (int k = 0; k < x.nreac; ++k) x.dnu -= x.reac_nu[k];
        x.npart = 0;
        auto part = [&](int sp) -> Part & {
            for (int k = 0; k < x.npart; ++k) if (x.part[k].sp == sp) return x.part[k];
            Part &p = x.part[x.npart++];
            p.sp = sp; p.nu_r = 0; p.nu_p = 0; p.nu = 0;
            return p;
        };
        for (int k = 0; k < x.nreac; ++k) part(x.reac_sp[k]).nu_r += x.reac_nu[k];
        for (int k = 0; k < x.nprod; ++k) part(x.prod_sp[k]).nu_p += x.prod_nu[k];
        for (int k = 0; k < x.npart; ++k) x.part[k].nu = x.part[k].nu_p - x.part[k].nu_r;
    }
    return KIN_OK;
}

// ------------------------------------------------------------------------------------------
// Code generation
// ------------------------------------------------------------------------------------------

static std::string lit(double v)
{
    char buf[64];
    std::snprintf(buf, sizeof buf, "%.17g", v);
    std::string s(buf);
    if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
    return "(" + s + ")";
}

// Constants of the generated code.  Values the hardware encodes for free in an instruction
// (small integers and a few powers of two) stay literals; every other FP64 constant goes to a
// per-mechanism table K[] read with scalar loads.  Literal FP64 constants would each need an
// SGPR pair, and hoisting hundreds of them out of the Newton loop exhausts the SGPRs.
struct Consts {
    std::vector<double> tab;
    std::map<uint64_t, int> index;
    std::string operator()(double v)
    {
        const double r = std::nearbyint(v);
        if ((r == v && v >= -16.0 && v <= 64.0) || v == 0.5 || v == -0.5 || v == 0.25 || v == -0.25)
            return lit(v);
        uint64_t bits;
        std::memcpy(&bits, &v, sizeof bits);
        auto it = index.find(bits);
        int k;
        if (it != index.end()) {
            k = it->second;
        } else {
            k = (int)tab.size();
            tab.push_back(v);
            index.emplace(bits, k);
        }
        return "K[" + std::to_string(k) + "]";
    }
};

// Horner form c[0] + T (c[1] + T (c[2] + ...)) with trailing zero coefficients dropped.
static std::string horner(const std::vector<std::string> &c, const std::vector<bool> &zero)
{
    int top = (int)c.size() - 1;
    while (top > 0 && zero[top]) --top;
    std::string e = c[top];
    for (int k = top - 1; k >= 0; --k) e = "fma(T, " + e + ", " + c[k] + ")";
    return e;
}

// NASA-7 species functions of species s at (T, iT, lT) into cp{s}, h{s} (h/RT, unless need_h
// is false and an earlier h{s} at the same T is in scope), s{s} (s/R), dc{s} (d(cp/R)/dT).
// With two different coefficient sets the set is selected by T < T_mid.
static void emit_thermo(std::ostringstream &o, Consts &K, const MechHost &m, int s, bool need_s,
                        bool need_dc, bool need_h = true)
{
    const double *lo = &m.nasa[14 * s], *hi = &m.nasa[14 * s + 7];
    const bool one = m.single_range(s);
    if (!one) o << "    const bool lo" << s << " = T < " << K(m.Tmid[s]) << ";\n";
    auto coef = [&](double vlo, double vhi) {
        if (one) return K(vlo);
        return "(lo" + std::to_string(s) + " ? " + K(vlo) + " : " + K(vhi) + ")";
    };
    auto is_zero = [&](int k) { return lo[k] == 0.0 && hi[k] == 0.0; };
    {
        std::vector<std::string> c; std::vector<bool> z;
        for (int k = 0; k < 5; ++k) { c.push_back(coef(lo[k], hi[k])); z.push_back(is_zero(k)); }
        o << "    const double cp" << s << " = " << horner(c, z) << ";\n";
    }
    if (need_h) {
        std::vector<std::string> c; std::vector<bool> z;
        for (int k = 0; k < 5; ++k) { c.push_back(coef(lo[k] / (k + 1), hi[k] / (k + 1))); z.push_back(is_zero(k)); }
        o << "    const double h" << s << " = fma(" << coef(lo[5], hi[5]) << ", iT, " << horner(c, z) << ");\n";
    }
    if (need_s) {
        std::vector<std::string> c; std::vector<bool> z;
        c.push_back(coef(lo[6], hi[6])); z.push_back(false);
        c.push_back(coef(lo[1], hi[1])); z.push_back(is_zero(1));
        for (int k = 2; k < 5; ++k) { c.push_back(coef(lo[k] / k, hi[k] / k)); z.push_back(is_zero(k)); }
        o << "    const double s" << s << " = fma(" << coef(lo[0], hi[0]) << ", lT, " << horner(c, z) << ");\n";
        o << "    const double g" << s << " = h" << s << " - s" << s << ";\n";
    }
    if (need_dc) {
        std::vector<std::string> c; std::vector<bool> z;
        for (int k = 1; k < 5; ++k) { c.push_back(coef(k * lo[k], k * hi[k])); z.push_back(is_zero(k)); }
        o << "    const double dc" << s << " = " << horner(c, z) << ";\n";
    }
}

static std::string cpow(int sp, int nu)
{
    std::string c = "c" + std::to_string(sp);
    std::string e = c;
    for (int k = 1; k < nu; ++k) e += " * " + c;
    return e;
}

// k * prod over (sp, nu) of c_sp^nu
static std::string mass_action(const std::string &k, const int *sp, const int *nu, int n)
{
    std::string e = k;
    for (int j = 0; j < n; ++j) e += " * " + cpow(sp[j], nu[j]);
    return e;
}

// d/dc_target of k * prod c^nu (empty string if the species is not on this side)
static std::string mass_action_grad(const std::string &k, const int *sp, const int *nu, int n, int target)
{
    int jt = -1;
    for (int j = 0; j < n; ++j) if (sp[j] == target) jt = j;
    if (jt < 0) return "";
    std::string e = k;
    if (nu[jt] > 1) e += " * " + lit((double)nu[jt]) + " * " + cpow(sp[jt], nu[jt] - 1);
    for (int j = 0; j < n; ++j) if (j != jt) e += " * " + cpow(sp[j], nu[j]);
    return e;
}

// e^x of the rate expressions (finite arguments: T is confined to [200, 6000] K).  Cody and
// Waite's reduction x = k ln2 + r, k = rint(x / ln2), |r| <= ln2 / 2, with ln2 split in a high
// part of 32 significant bits (k * hi exact for |k| < 2^21) and the rest; e^r by its Taylor
// polynomial to degree 12 (truncation below 2.3e-16 relative), then 2^k by ldexp, which gives
// infinity or zero beyond the double range.  About two ulp, in 18 instructions.
static const char *kLaneExp =
    "__device__ __forceinline__ double kin_exp(double x)\n{\n"
    "    const double k = rint(x * 1.4426950408889634);\n"
    "    double r = fma(-k, 0x1.62e42fee00000p-1, x);\n"
    "    r = fma(-k, 0x1.a39ef35793c76p-33, r);\n"
    "    double p = 1.0 / 479001600.0;\n"
    "    p = fma(p, r, 1.0 / 39916800.0);\n"
    "    p = fma(p, r, 1.0 / 3628800.0);\n"
    "    p = fma(p, r, 1.0 / 362880.0);\n"
    "    p = fma(p, r, 1.0 / 40320.0);\n"
    "    p = fma(p, r, 1.0 / 5040.0);\n"
    "    p = fma(p, r, 1.0 / 720.0);\n"
    "    p = fma(p, r, 1.0 / 120.0);\n"
    "    p = fma(p, r, 1.0 / 24.0);\n"
    "    p = fma(p, r, 1.0 / 6.0);\n"
    "    p = fma(p, r, 0.5);\n"
    "    p = fma(p, r, 1.0);\n"
    "    p = fma(p, r, 1.0);\n"
    "    return ldexp(p, (int)k);\n}\n\n";

std::string lane_source(const MechHost &m, int block, std::vector<double> &consts)
{
    const int ns = m.ns;
    Consts K;
    std::ostringstream o;

    // --- f and J -----------------------------------------------------------------------------
    o << "__device__ __forceinline__ void kin_eval(kin_cptr K, const double rho, "
         "const double (&x)[KIN_N], double (&f)[KIN_N], double (&J)[KIN_N][KIN_N])\n{\n";
    o << "    const double T = x[KIN_NS];\n    const double iT = 1.0 / T;\n    const double lT = log(T);\n";
    o << "    const double rc = 1e-3 * rho;\n    const double irc = 1.0 / rc;\n";
    o << "    const double lPaRT = " << K(std::log(kPatmCgs / kRuCgs)) << " - lT;\n";
    for (int s = 0; s < ns; ++s) emit_thermo(o, K, m, s, true, false);
    for (int s = 0; s < ns; ++s)
        o << "    const double c" << s << " = x[" << s << "] * (rc * " << K(1.0 / m.M[s]) << ");\n";
    // f[s] and the species rows of J accumulate over the reactions; an entry's first term is
    // assigned, not added to a zero.  The species-by-species block accumulates sum_r nu dq_r,
    // and the mass ratios M_s / M_k are applied once after the reactions, so the reaction
    // blocks need no per-entry constants.
    std::vector<bool> f_set(ns, false), J_set((size_t)ns * (ns + 1), false);
    auto accum = [&](const std::string &dst, bool &set, const std::string &coef, const std::string &v) {
        if (!set) {
            if (coef == "1.0") o << "        " << dst << " = " << v << ";\n";
            else if (coef == "-1.0") o << "        " << dst << " = -" << v << ";\n";
            else o << "        " << dst << " = " << coef << " * " << v << ";\n";
            set = true;
        } else {
            o << "        " << dst << " = fma(" << coef << ", " << v << ", " << dst << ");\n";
        }
    };
    for (int r = 0; r < m.nr; ++r) {
        const Rxn &x = m.rx[r];
        o << "    { // reaction " << r << "\n";
        o << "        K = kin_fence_k(K);\n";
        std::string lk = K(x.lnA);
        if (x.b != 0.0) lk = "fma(" + K(x.b) + ", lT, " + lk + ")";
        if (x.Ta != 0.0) lk = "fma(" + K(-x.Ta) + ", iT, " + lk + ")";
        o << "        const double lkf = " << lk << ";\n";
        o << "        const double kf = kin_exp(lkf);\n";
        o << "        const double dlkf = " << ((x.b != 0.0 || x.Ta != 0.0) ? "fma(" + K(x.Ta) + ", iT, " + K(x.b) + ") * iT" : std::string("0.0")) << ";\n";
        o << "        const double pf = " << mass_action("kf", x.reac_sp, x.reac_nu, x.nreac) << ";\n";
        if (x.rev) {
            // sums of nu_s g_s and nu_s h_s: the first term stands alone (a literal zero to
            // start from would cost an add, since 0 + (-0) is not -0), and a zero change of
            // moles drops its term
            std::string sg, sh;
            auto term = [&](int nu, const std::string &v) {
                return nu == 1 ? v : nu == -1 ? "(-" + v + ")" : "(" + lit((double)nu) + " * " + v + ")";
            };
            for (int k = 0; k < x.npart; ++k) {
                const int nu = x.part[k].nu;
                if (!nu) continue;
                const std::string g = "g" + std::to_string(x.part[k].sp), h = "h" + std::to_string(x.part[k].sp);
                sg = sg.empty() ? term(nu, g) : "fma(" + lit((double)nu) + ", " + g + ", " + sg + ")";
                sh = sh.empty() ? term(nu, h) : "fma(" + lit((double)nu) + ", " + h + ", " + sh + ")";
            }
            if (sg.empty()) sg = sh = "0.0";
            if (x.dnu != 0)
                o << "        const double lKc = " << lit((double)x.dnu) << " * lPaRT - " << sg << ";\n";
            else
                o << "        const double lKc = -" << sg << ";\n";
            o << "        const double kb = kin_exp(lkf - lKc);\n";
            if (x.dnu != 0)
                o << "        const double dlKc = (" << lit((double)-x.dnu) << " + " << sh << ") * iT;\n";
            else
                o << "        const double dlKc = " << sh << " * iT;\n";
            o << "        const double pb = " << mass_action("kb", x.prod_sp, x.prod_nu, x.nprod) << ";\n";
            o << "        const double D = pf - pb;\n";
        } else {
            o << "        const double D = pf;\n";
        }
        std::string Mfac = "";
        if (x.tb >= 0) {
            std::string e = "0.0";
            for (int s = 0; s < ns; ++s) {
                double a = m.eff[(size_t)x.tb * ns + s];
                if (a != 0.0) e = "fma(" + K(a) + ", c" + std::to_string(s) + ", " + e + ")";
            }
            o << "        const double Mc = " << e << ";\n";
            Mfac = "Mc * ";
        }
        o << "        const double q = " << Mfac << "D;\n";
        if (x.rev)
            o << "        const double dqT = " << Mfac << "(pf * dlkf - pb * (dlkf - dlKc));\n";
        else
            o << "        const double dqT = " << Mfac << "(pf * dlkf);\n";
        bool has_dq[6] = {false, false, false, false, false, false};
        for (int k = 0; k < x.npart; ++k) {
            const int sp = x.part[k].sp;
            std::string gf = mass_action_grad("kf", x.reac_sp, x.reac_nu, x.nreac, sp);
            std::string gb = x.rev ? mass_action_grad("kb", x.prod_sp, x.prod_nu, x.nprod, sp) : "";
            std::string e;
            if (!gf.empty() && !gb.empty()) e = "(" + gf + " - " + gb + ")";
            else if (!gf.empty()) e = "(" + gf + ")";
            else if (!gb.empty()) e = "(-(" + gb + "))";
            if (e.empty()) continue;
            has_dq[k] = true;
            o << "        const double dq" << k << " = " << Mfac << e << ";\n";
        }
        // f[s] accumulates the molar production and J[s][NS] the rate's T-derivative; both
        // are scaled by M_s / rho_cgs after the reaction loop.
        for (int a = 0; a < x.npart; ++a) {
            const Part &p = x.part[a];
            if (!p.nu) continue;
            const int s = p.sp;
            const double nu = (double)p.nu;
            {
                bool fs = f_set[s];
                accum("f[" + std::to_string(s) + "]", fs, lit(nu), "q");
                f_set[s] = fs;
            }
            auto jref = [&](int k) { return J_set[(size_t)s * (ns + 1) + k]; };
            {
                bool js = jref(ns);
                accum("J[" + std::to_string(s) + "][KIN_NS]", js, lit(nu), "dqT");
                J_set[(size_t)s * (ns + 1) + ns] = js;
            }
            for (int k = 0; k < x.npart; ++k) {
                if (!has_dq[k]) continue;
                const int sk = x.part[k].sp;
                bool js = jref(sk);
                accum("J[" + std::to_string(s) + "][" + std::to_string(sk) + "]", js, lit(nu), "dq" + std::to_string(k));
                J_set[(size_t)s * (ns + 1) + sk] = js;
            }
            if (x.tb >= 0) {
                for (int k = 0; k < ns; ++k) {
                    double a2 = m.eff[(size_t)x.tb * ns + k];
                    if (a2 == 0.0) continue;
                    bool js = jref(k);
                    accum("J[" + std::to_string(s) + "][" + std::to_string(k) + "]", js, K(nu * a2), "D");
                    J_set[(size_t)s * (ns + 1) + k] = js;
                }
            }
        }
        o << "    }\n";
    }
    for (int s = 0; s < ns; ++s) {
        if (!f_set[s]) o << "    f[" << s << "] = 0.0;\n";
        for (int k = 0; k <= ns; ++k)
            if (!J_set[(size_t)s * (ns + 1) + k]) o << "    J[" << s << "][" << k << "] = 0.0;\n";
    }
    // species rows of f, temperature column, energy row
    for (int s = 0; s < ns; ++s) {
        o << "    {\n        const double ms = " << K(m.M[s]) << " * irc;\n";
        o << "        f[" << s << "] *= ms;\n        J[" << s << "][KIN_NS] *= ms;\n";
        for (int k = 0; k < ns; ++k)
            if (k != s && J_set[(size_t)s * (ns + 1) + k])
                o << "        J[" << s << "][" << k << "] *= " << K(m.M[s] / m.M[k]) << ";\n";
        o << "    }\n";
    }
    o << "    double cv = 0.0, dcv = 0.0, de = 0.0;\n";
    o << "    double ek[KIN_NS], cvk[KIN_NS];\n";
    for (int s = 0; s < ns; ++s) {
        o << "    {\n";
        emit_thermo(o, K, m, s, false, true, false);   // h_s from the first pass
        const double rm = kRu * 1e3 / m.M[s];
        o << "    ek[" << s << "] = " << K(rm) << " * T * (h" << s << " - 1.0);\n";
        o << "    cvk[" << s << "] = " << K(rm) << " * (cp" << s << " - 1.0);\n";
        o << "    cv = fma(x[" << s << "], cvk[" << s << "], cv);\n";
        o << "    dcv = fma(x[" << s << "], " << K(rm) << " * dc" << s << ", dcv);\n";
        o << "    de = fma(ek[" << s << "], f[" << s << "], de);\n";
        o << "    }\n";
    }
    o << "    const double fT = -de / cv;\n    f[KIN_NS] = fT;\n    const double icv = 1.0 / cv;\n";
    o << "#pragma unroll\n    for (int k = 0; k < KIN_NS; ++k) {\n        double acc = 0.0;\n"
         "#pragma unroll\n        for (int s = 0; s < KIN_NS; ++s) acc = fma(ek[s], J[s][k], acc);\n"
         "        J[KIN_NS][k] = -fma(fT, cvk[k], acc) * icv;\n    }\n";
    o << "    {\n        double acc = 0.0;\n#pragma unroll\n        for (int s = 0; s < KIN_NS; ++s) "
         "acc = fma(cvk[s], f[s], fma(ek[s], J[s][KIN_NS], acc));\n"
         "        J[KIN_NS][KIN_NS] = -fma(fT, dcv, acc) * icv;\n    }\n";
    o << "}\n\n";

    // --- e(Y, T) and c_v ------------------------------------------------------------------------
    o << "__device__ __forceinline__ void kin_energy_cv(kin_cptr K, "
         "const double (&x)[KIN_N], const double T, double &e, double &cv)\n{\n";
    o << "    const double iT = 1.0 / T;\n    e = 0.0;\n    cv = 0.0;\n";
    for (int s = 0; s < ns; ++s) {
        o << "    {\n";
        emit_thermo(o, K, m, s, false, false);
        const double rm = kRu * 1e3 / m.M[s];
        o << "        e = fma(x[" << s << "], " << K(rm) << " * T * (h" << s << " - 1.0), e);\n";
        o << "        cv = fma(x[" << s << "], " << K(rm) << " * (cp" << s << " - 1.0), cv);\n";
        o << "    }\n";
    }
    o << "}\n\n";

    std::ostringstream head;
    head << "// generated for a mechanism of " << ns << " species and " << m.nr << " reactions\n";
    head << "#define KIN_NS " << ns << "\n#define KIN_N " << ns + 1 << "\n#define KIN_BLOCK " << block
         << "\n#define KIN_NCONST " << K.tab.size() << "\n";
    head << "typedef const __attribute__((address_space(4))) double *kin_cptr;  // scalar-loaded constants\n";
    head << "// Opaque copy of the table pointer: loads of K[] cannot move above it, which keeps the\n"
            "// scalar loads of each reaction's constants next to that reaction.\n"
            "__device__ __forceinline__ kin_cptr kin_fence_k(kin_cptr p)\n{\n"
            "    asm volatile(\"\" : \"+s\"(p));\n    return p;\n}\n\n";
    head << kLaneExp;
    consts = K.tab;
    // the launch passes the host's AdvanceArgs by value as the kernel's KinLaneArgs
    std::ostringstream tail;
    tail << "\nstatic_assert(sizeof(KinLaneArgs) == " << sizeof(AdvanceArgs)
         << ", \"KinLaneArgs must mirror the host launch arguments\");\n";
    return head.str() + o.str() + kLaneTemplate + tail.str();
}

kin_status rtc_compile(const std::string &src, const char *name, std::vector<char> &code,
                       std::string &msg, double *seconds)
{
    auto t0 = std::chrono::steady_clock::now();
    if (const char *dump = std::getenv("KIN_JIT_DUMP")) {  // write the generated source
        if (FILE *f = std::fopen(dump, "w")) {
            std::fwrite(src.data(), 1, src.size(), f);
            std::fclose(f);
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), name, 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        msg = "hiprtcCreateProgram failed";
        return KIN_ECOMPILE;
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-mllvm", "-pragma-unroll-threshold=1000000"};
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string log(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &log[0]);
    if (rc != HIPRTC_SUCCESS) {
        msg = std::string("hipRTC compile failed: ") + hiprtcGetErrorString(rc) + "\n" + log;
        hiprtcDestroyProgram(&prog);
        return KIN_ECOMPILE;
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    msg = log;
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return KIN_OK;
}

}  // namespace kin
