// kin_global.hip -- the global-memory tier, for mechanisms beyond the wave layout's 63 species
// (up to 255).  It follows the first of the paper's two kinetics kernels (Sec. 4.2): one
// thread per cell, the cell's whole Jacobian in global memory, stored entry-major so that the
// 64 cells of a wavefront touch one entry in one coalesced access.  Gaussian elimination with
// partial pivoting streams the matrix through memory, so this tier is bound by HBM bandwidth,
// not by the vector ALUs.  The working set of a launch (matrix, vectors) lives in a workspace
// of S slots, one per thread; a cell occupies a slot from its first to its last Newton
// iteration, and a slot that finishes its cell takes the next one from the work counter.
//
// Method as in the other layouts: Newton iterations on backward Euler in x = (Y, T) for a
// constant-(rho, e) cell, (I - hJ) dx = -G, dyadic sub-step halving on failure (Sec. 3.2,
// Eq. "kinetics"; energy bookkeeping of Sec. 2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kin_internal.h"

namespace kin {
namespace {

constexpr double gTmin = 200.0, gTmax = 6000.0;
constexpr int kGRows = 8;  // rows eliminated per pass of the pivot row

// Workspace of S slots, entry-major: entry e of slot s sits at base[e * S + s].
struct GWork {
    double *J;   // [N * N]  Jacobian, then the Newton matrix and its LU factors
    double *f;   // [N]      production sums, then f, then the right-hand side and the update
    double *x;   // [N]      last accepted state
    double *xk;  // [N]      Newton iterate
    double *c;   // [ns]     concentrations
    double *g;   // [ns]     g/RT, then e_s
    double *hh;  // [ns]     h/RT, then c_v,s
    double *Mc;  // [ntb]    third-body concentrations, then q_f - q_b of the slot's reaction
    long long S;
};

__device__ __forceinline__ GWork gwork_map(double *base, int ns, int ntb, long long S)
{
    const size_t N = (size_t)ns + 1;
    GWork w;
    double *p = base;
    w.J = p; p += N * N * (size_t)S;
    w.f = p; p += N * (size_t)S;
    w.x = p; p += N * (size_t)S;
    w.xk = p; p += N * (size_t)S;
    w.c = p; p += (size_t)ns * S;
    w.g = p; p += (size_t)ns * S;
    w.hh = p; p += (size_t)ns * S;
    w.Mc = p;
    w.S = S;
    return w;
}

struct GThermo {
    double cp, h, s, dcp;
};

// NASA-7 functions of species s at T: cp/R, h/RT, s/R and d(cp/R)/dT.
__device__ __forceinline__ GThermo gthermo(const WaveTables &t, int s, double T, double iT, double lT)
{
    const double *a = t.nasa + 14 * s + (T < t.Tmid[s] ? 0 : 7);
    GThermo o;
    o.cp = fma(T, fma(T, fma(T, fma(T, a[4], a[3]), a[2]), a[1]), a[0]);
    o.h = fma(a[5], iT, fma(T, fma(T, fma(T, fma(T, a[4] * 0.2, a[3] * 0.25), a[2] * (1.0 / 3.0)), a[1] * 0.5), a[0]));
    o.s = fma(a[0], lT, fma(T, fma(T, fma(T, fma(T, a[4] * 0.25, a[3] * (1.0 / 3.0)), a[2] * 0.5), a[1]), a[6]));
    o.dcp = fma(T, fma(T, fma(T, 4.0 * a[4], 3.0 * a[3]), 2.0 * a[2]), a[1]);
    return o;
}

// c^|nu| and its derivative for nu in 0..3, branch-free.
__device__ __forceinline__ void gpow(double c, int nu, double &p, double &dp)
{
    const double h = (nu >= 2 ? c : 1.0) * (nu >= 3 ? c : 1.0);
    p = (nu >= 1 ? c : 1.0) * h;
    dp = (double)nu * h;
}

// Mixture e (J/kg) and c_v (J/kg/K) of slot `sl`'s iterate at T.
__device__ __forceinline__ void genergy(const WaveTables &t, const GWork &w, long long sl, double T,
                                       double &e, double &cv)
{
    e = 0.0;
    cv = 0.0;
    const double iT = 1.0 / T;
    for (int s = 0; s < t.ns; ++s) {
        const GThermo th = gthermo(t, s, T, iT, 0.0);
        const double rm = 8.31446261815324e3 / t.M[s];
        const double y = w.xk[(size_t)s * w.S + sl];
        e = fma(y, rm * T * (th.h - 1.0), e);
        cv = fma(y, rm * (th.cp - 1.0), cv);
    }
}

__device__ bool ginvert_T(const WaveTables &t, const GWork &w, long long sl, double e0, double T0,
                          double &T_out)
{
    double T = T0;
    for (int it = 0; it < 20; ++it) {
        double e, cv;
        genergy(t, w, sl, T, e, cv);
        if (!(cv > 0.0)) break;
        const double dT = (e - e0) / cv;
        T -= dT;
        if (!__builtin_isfinite(T) || T < gTmin || T > gTmax) break;
        if (fabs(dT) <= 1e-13 * T) { T_out = T; return true; }
    }
    double lo = gTmin, hi = gTmax, e, cv;
    genergy(t, w, sl, lo, e, cv);
    const double flo = e - e0;
    genergy(t, w, sl, hi, e, cv);
    const double fhi = e - e0;
    if (!(flo <= 0.0 && fhi >= 0.0)) return false;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * lo; ++it) {
        const double mid = 0.5 * (lo + hi);
        genergy(t, w, sl, mid, e, cv);
        if (e - e0 > 0.0) hi = mid; else lo = mid;
    }
    T_out = 0.5 * (lo + hi);
    return true;
}

// f = dx/dt into w.f and J = df/dx into w.J at the iterate w.xk.
__device__ void geval(const WaveTables &t, const GWork &w, long long sl, double rho)
{
    const int ns = t.ns, N = ns + 1;
    const size_t S = (size_t)w.S;
    double *J = w.J + sl, *f = w.f + sl;
    const auto Jat = [&](int i, int j) -> double & { return J[((size_t)i * N + j) * S]; };
    const double T = w.xk[(size_t)ns * S + sl];
    const double iT = 1.0 / T, lT = log(T);
    const double rc = 1e-3 * rho, irc = 1.0 / rc;
    const double lPaRT = t.lnPaR - lT;
    for (int s = 0; s < ns; ++s) {
        const GThermo th = gthermo(t, s, T, iT, lT);
        w.c[(size_t)s * S + sl] = w.xk[(size_t)s * S + sl] * (rc / t.M[s]);
        w.g[(size_t)s * S + sl] = th.h - th.s;
        w.hh[(size_t)s * S + sl] = th.h;
    }
    for (size_t e = 0; e < (size_t)N * N; ++e) J[e * S] = 0.0;
    for (int i = 0; i < N; ++i) f[(size_t)i * S] = 0.0;
    // third-body concentrations [M]_q = sum_s eff_qs c_s
    for (int q = 0; q < t.ntb; ++q) {
        double acc = 0.0;
        for (int s = 0; s < ns; ++s) acc = fma(t.effT[(size_t)s * t.ntb + q], w.c[(size_t)s * S + sl], acc);
        w.Mc[(size_t)q * S + sl] = acc;
    }
    // reactions: Q_r = [M]_r (k_f prod c^nu' - k_b prod c^nu''), six species slots per
    // reaction (reactants 0-2, products 3-5, unused slots have nu = 0)
    const double4 *rxd4 = reinterpret_cast<const double4 *>(t.rxd);
    for (int r = 0; r < t.nr; ++r) {
        const RxnRec x = t.rxc[r];
        const double4 rd = rxd4[r];
        const RxnCoef *kc = t.rxk + r;
        const double lkf = fma(-rd.z, iT, fma(rd.y, lT, rd.x));
        const double kf = exp(lkf);
        const double dlkf = fma(rd.z, iT, rd.y) * iT;
        double pw[6], dpw[6], sg = 0.0, sh = 0.0;
        int sp[6];
        for (int q = 0; q < 6; ++q) {
            sp[q] = x.coff[q] >> 3;
            double cq = 1.0;
            if (x.nu[q] != 0) {
                cq = w.c[(size_t)sp[q] * S + sl];
                sg = fma((double)x.nu[q], w.g[(size_t)sp[q] * S + sl], sg);
                sh = fma((double)x.nu[q], w.hh[(size_t)sp[q] * S + sl], sh);
            }
            gpow(cq, q < 3 ? -x.nu[q] : x.nu[q], pw[q], dpw[q]);
        }
        const double pf = kf * (pw[0] * pw[1] * pw[2]);
        double dq[6];
        dq[0] = kf * (dpw[0] * pw[1] * pw[2]);
        dq[1] = kf * (pw[0] * dpw[1] * pw[2]);
        dq[2] = kf * (pw[0] * pw[1] * dpw[2]);
        const double lKc = rd.w * lPaRT - sg;
        const double kb = exp(lkf - lKc);
        const double dlKc = (sh - rd.w) * iT;
        const bool rev = x.rev != 0;
        const double pb = rev ? kb * (pw[3] * pw[4] * pw[5]) : 0.0;
        dq[3] = rev ? -kb * (dpw[3] * pw[4] * pw[5]) : 0.0;
        dq[4] = rev ? -kb * (pw[3] * dpw[4] * pw[5]) : 0.0;
        dq[5] = rev ? -kb * (pw[3] * pw[4] * dpw[5]) : 0.0;
        const double Mc = x.tb >= 0 ? w.Mc[(size_t)x.tb * S + sl] : 1.0;
        const double D = pf - pb;
        const double q = Mc * D;
        const double qT = Mc * (pf * dlkf - pb * (dlkf - dlKc));
        if (x.tb >= 0) w.Mc[(size_t)x.tb * S + sl] = D;
        for (int k = 0; k < 6; ++k) dq[k] = Mc * dq[k] * kc->colc[k];
        for (int i = 0; i < 6; ++i) {
            if (x.nu[i] == 0) continue;
            const double nu = (double)x.nu[i];
            const double a = kc->rowc[i];
            f[(size_t)sp[i] * S] += nu * q;
            Jat(sp[i], ns) += nu * qT;
            for (int j = 0; j < 6; ++j)
                if (x.nu[j] != 0) Jat(sp[i], sp[j]) += a * dq[j];
        }
    }
    // dense third-body terms: J[s][k] += D_q nu_qs M_s eff_qk / M_k
    for (int e = 0; e < t.ntbe; ++e) {
        const int ent = t.tbe[e];
        const double D = w.Mc[(size_t)(ent & 0xffff) * S + sl];
        const int row = ent >> 16;
        const double *er = t.effR + (size_t)e * ns;
        for (int k = 0; k < ns; ++k) Jat(row, k) += D * er[k];
    }
    // species rows of f and the temperature column; e_s and c_v,s replace g and h
    double cv = 0.0, dcv = 0.0, de = 0.0;
    for (int s = 0; s < ns; ++s) {
        const GThermo th = gthermo(t, s, T, iT, lT);
        const double rm = 8.31446261815324e3 / t.M[s];
        const double ms = t.M[s] * irc;
        const double fs = f[(size_t)s * S] * ms;
        f[(size_t)s * S] = fs;
        Jat(s, ns) *= ms;
        const double ek = rm * T * (th.h - 1.0), cvk = rm * (th.cp - 1.0);
        w.g[(size_t)s * S + sl] = ek;
        w.hh[(size_t)s * S + sl] = cvk;
        const double xs = w.xk[(size_t)s * S + sl];
        cv = fma(xs, cvk, cv);
        dcv = fma(xs, rm * th.dcp, dcv);
        de = fma(ek, fs, de);
    }
    const double fT = -de / cv, icv = 1.0 / cv;
    // energy row: J[ns][k] = -(sum_s e_s J[s][k] + f_T c_v,k) / c_v
    for (int k = 0; k < ns; ++k) {
        double acc = 0.0;
        for (int s = 0; s < ns; ++s) acc = fma(w.g[(size_t)s * S + sl], Jat(s, k), acc);
        Jat(ns, k) = -fma(fT, w.hh[(size_t)k * S + sl], acc) * icv;
    }
    double acc = 0.0;
    for (int s = 0; s < ns; ++s)
        acc = fma(w.hh[(size_t)s * S + sl], f[(size_t)s * S], fma(w.g[(size_t)s * S + sl], Jat(s, ns), acc));
    Jat(ns, ns) = -fma(fT, dcv, acc) * icv;
    f[(size_t)ns * S] = fT;
}

// Gaussian elimination with partial pivoting (first row of largest |a_ik|) on the slot's
// Newton matrix, applied to the right-hand side in w.f, then back substitution: w.f holds the
// update on return.  Rows are exchanged in memory.  F32: the factorisation and solves run in
// FP32 on values rounded from the FP64 matrix (already row-equilibrated by the caller).
template <bool F32>
__device__ bool glu_solve(const GWork &w, long long sl, int N)
{
    using R = typename std::conditional<F32, float, double>::type;
    const size_t S = (size_t)w.S;
    double *A = w.J + sl, *b = w.f + sl;
    const auto Aat = [&](int i, int j) -> double & { return A[((size_t)i * N + j) * S]; };
    for (int k = 0; k < N; ++k) {
        int p = k;
        R amax = (R)fabs((R)Aat(k, k));
        for (int i = k + 1; i < N; ++i) {
            const R v = (R)fabs((R)Aat(i, k));
            if (v > amax) { amax = v; p = i; }
        }
        if (amax == R(0)) return false;
        if (p != k) {
            for (int j = k; j < N; ++j) {
                const double tk = Aat(k, j);
                Aat(k, j) = Aat(p, j);
                Aat(p, j) = tk;
            }
            const double tb = b[(size_t)k * S];
            b[(size_t)k * S] = b[(size_t)p * S];
            b[(size_t)p * S] = tb;
        }
        const R piv = (R)Aat(k, k);
        const R yk = (R)b[(size_t)k * S];
        // rows in groups of kGRows: each pivot-row element is loaded once per group, and the
        // group's loads per column pair are independent, which keeps enough memory operations
        // in flight per thread
        int i = k + 1;
        for (; i + kGRows <= N; i += kGRows) {
            R l[kGRows];
#pragma unroll
            for (int r = 0; r < kGRows; ++r) l[r] = (R)Aat(i + r, k) / piv;
            int j = k + 1;
            for (; j + 2 <= N; j += 2) {
                const R a0 = (R)Aat(k, j), a1 = (R)Aat(k, j + 1);
                R v[kGRows][2];
#pragma unroll
                for (int r = 0; r < kGRows; ++r) { v[r][0] = (R)Aat(i + r, j); v[r][1] = (R)Aat(i + r, j + 1); }
#pragma unroll
                for (int r = 0; r < kGRows; ++r) {
                    Aat(i + r, j) = (double)fma(-l[r], a0, v[r][0]);
                    Aat(i + r, j + 1) = (double)fma(-l[r], a1, v[r][1]);
                }
            }
            for (; j < N; ++j) {
                const R a0 = (R)Aat(k, j);
#pragma unroll
                for (int r = 0; r < kGRows; ++r) Aat(i + r, j) = (double)fma(-l[r], a0, (R)Aat(i + r, j));
            }
#pragma unroll
            for (int r = 0; r < kGRows; ++r) b[(size_t)(i + r) * S] = (double)fma(-l[r], yk, (R)b[(size_t)(i + r) * S]);
        }
        for (; i < N; ++i) {
            const R l = (R)Aat(i, k) / piv;
            for (int j = k + 1; j < N; ++j) Aat(i, j) = (double)fma(-l, (R)Aat(k, j), (R)Aat(i, j));
            b[(size_t)i * S] = (double)fma(-l, yk, (R)b[(size_t)i * S]);
        }
    }
    for (int i = N - 1; i >= 0; --i) {
        R s = (R)b[(size_t)i * S];
        for (int j = i + 1; j < N; ++j) s = fma(-(R)Aat(i, j), (R)b[(size_t)j * S], s);
        b[(size_t)i * S] = (double)(s / (R)Aat(i, i));
    }
    return true;
}

enum { G_CONTINUE = 0, G_ACCEPTED = 1, G_FAILED = 2 };

// One Newton iteration of slot sl on the backward-Euler system of sub-step h.
template <bool F32>
__device__ int gnewton(const WaveTables &t, const AdvanceArgs &a, const GWork &w, long long sl, double rho,
                       double e0, double h, double &r_prev)
{
    const int ns = t.ns, N = ns + 1;
    const size_t S = (size_t)w.S;
    geval(t, w, sl, rho);
    double *A = w.J + sl, *b = w.f + sl;
    double chk = 0.0;
    for (int i = 0; i < N; ++i) {
        const double gi = -((w.xk[(size_t)i * S + sl] - w.x[(size_t)i * S + sl]) - h * b[(size_t)i * S]);
        double m = 0.0;
        for (int j = 0; j < N; ++j) {
            double &aij = A[((size_t)i * N + j) * S];
            const double v = (i == j ? 1.0 : 0.0) - h * aij;
            aij = v;
            chk += v - v;
            m = fmax(m, fabs(v));
        }
        chk += gi - gi;
        if (F32) {  // row equilibration before rounding to FP32
            const double sc = 1.0 / m;
            for (int j = 0; j < N; ++j) A[((size_t)i * N + j) * S] *= sc;
            b[(size_t)i * S] = gi * sc;
        } else {
            b[(size_t)i * S] = gi;
        }
    }
    if (!(chk == 0.0)) return G_FAILED;
    if (!glu_solve<F32>(w, sl, N)) return G_FAILED;
    bool conv = true;
    double chk2 = 0.0, r = 0.0;
    for (int i = 0; i < N; ++i) {
        const double d = b[(size_t)i * S];
        const double xi = w.xk[(size_t)i * S + sl] + d;
        w.xk[(size_t)i * S + sl] = xi;
        chk2 += xi - xi;
        const double atol = (i < ns) ? a.atol_Y : a.atol_T;
        conv = conv && (fabs(d) <= atol + a.rtol * fabs(xi));
        r = fmax(r, fabs(d) / (atol + a.rtol * fabs(xi)));
    }
    if (!(chk2 == 0.0)) return G_FAILED;
    const double Tk = w.xk[(size_t)ns * S + sl];
    if (Tk < gTmin || Tk > gTmax) return G_FAILED;
    if (!conv && !a.point_implicit) {
        if (a.diverge_ratio > 0.0) {
            if (r_prev >= 0.0 && r > a.diverge_ratio * r_prev) return G_FAILED;
            r_prev = r;
        }
        return G_CONTINUE;
    }
    if (!a.point_implicit)
        for (int s = 0; s < ns; ++s)
            if (w.xk[(size_t)s * S + sl] < -a.y_neg) return G_FAILED;
    double Tn;
    if (!ginvert_T(t, w, sl, e0, Tk, Tn)) return G_FAILED;
    w.xk[(size_t)ns * S + sl] = Tn;
    return G_ACCEPTED;
}

// Persistent slots: every loop trip performs one Newton iteration for the cell each thread
// holds; a thread that finishes its cell stores it and takes the next cell index from the
// work counter.  Controller as in the other layouts (dyadic sub-steps, halving on failure).
template <bool F32>
__global__ void __launch_bounds__(64) global_kernel(WaveTables t, AdvanceArgs a, double *wsbase, long long S)
{
    const long long sl = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= S) return;
    const GWork w = gwork_map(wsbase, t.ns, t.ntb, S);
    const int ns = t.ns, N = ns + 1;
    const bool adapt = a.L_forced < 0;
    const int Lc = adapt ? a.L_max : a.L_forced;
    const unsigned long long end = 1ull << Lc;
    for (;;) {
        const unsigned long long gi = atomicAdd(a.counter, 1ull);
        if (gi >= (unsigned long long)a.total) break;
        int j = 0;
        while (j + 1 < a.nspan && (unsigned long long)a.span[j + 1].start <= gi) ++j;
        const long long cell = (long long)gi - a.span[j].start;
        const double dt = a.span[j].dt;
        const Arena ar = arena_at(a.span[j].base, a.span[j].n, ns);
        const long long ld = a.span[j].n;
        const double rho = ar.rho[cell], e0 = ar.e0[cell];
        double chk = rho - rho + e0 - e0 + dt - dt;
        for (int s = 0; s < N; ++s) {
            const double v = (s < ns) ? ar.Y[(size_t)s * ld + cell] : ar.T[cell];
            w.x[(size_t)s * w.S + sl] = v;
            w.xk[(size_t)s * w.S + sl] = v;
            chk += v - v;
        }
        const double T0 = ar.T[cell];
        if (!(chk == 0.0) || !(rho > 0.0) || !(dt >= 0.0) || T0 < gTmin || T0 > gTmax) {
            ar.status[cell] = 3;
            ar.level[cell] = 0;
            ar.iters[cell] = 0;
            ar.sched[cell] = 0xcbf29ce484222325ull;
            continue;
        }
        unsigned long long tt = 0, hsh = 0xcbf29ce484222325ull;
        int l = adapt ? 0 : a.L_forced, level = l, iters = 0, k = 0, st = -1;
        bool failed = false;
        double r_prev = -1.0;
        while (st < 0) {
            if (k == 0 && iters >= a.max_iters) { st = 2; break; }
            ++iters;
            if (k == 0) r_prev = -1.0;
            int outcome = gnewton<F32>(t, a, w, sl, rho, e0, ldexp(dt, -l), r_prev);
            if (outcome == G_CONTINUE && ++k >= a.k_max) outcome = G_FAILED;
            if (outcome == G_CONTINUE) continue;
            hsh = (hsh ^ (unsigned long long)(2 * l + (outcome == G_ACCEPTED ? 1 : 0))) * 0x100000001b3ull;
            k = 0;
            if (outcome == G_ACCEPTED) {
                for (int s = 0; s < N; ++s) w.x[(size_t)s * w.S + sl] = w.xk[(size_t)s * w.S + sl];
                tt += 1ull << (Lc - l);
                if (adapt && l > 0 && (tt & ((1ull << (Lc - l + 1)) - 1ull)) == 0ull) --l;
                if (tt >= end) st = failed ? 1 : 0;
            } else {
                for (int s = 0; s < N; ++s) w.xk[(size_t)s * w.S + sl] = w.x[(size_t)s * w.S + sl];
                if (!adapt) {
                    st = 2;
                } else {
                    failed = true;
                    ++l;
                    if (l > level) level = l;
                    if (l > a.L_max) { level = a.L_max; st = 2; }
                }
            }
        }
        if (st < 2) {
            for (int s = 0; s < ns; ++s) ar.Y[(size_t)s * ld + cell] = w.x[(size_t)s * w.S + sl];
            ar.T[cell] = w.x[(size_t)ns * w.S + sl];
        }
        ar.status[cell] = st;
        ar.level[cell] = level;
        ar.iters[cell] = iters;
        ar.sched[cell] = hsh;
    }
}

}  // namespace

size_t global_work_doubles_per_slot(int ns, int ntb)
{
    const size_t N = (size_t)ns + 1;
    return N * N + 3 * N + 3 * (size_t)ns + (size_t)(ntb > 0 ? ntb : 1);
}

hipError_t launch_global(const WaveTables &t, const AdvanceArgs &a, bool f32, double *work, long long slots,
                         hipStream_t s)
{
    if (slots <= 0) return hipSuccess;
    const int block = 64;
    const long long grid = (slots + block - 1) / block;
    if (f32)
        hipLaunchKernelGGL((global_kernel<true>), dim3((unsigned)grid), dim3(block), 0, s, t, a, work, slots);
    else
        hipLaunchKernelGGL((global_kernel<false>), dim3((unsigned)grid), dim3(block), 0, s, t, a, work, slots);
    return hipGetLastError();
}

}  // namespace kin
