// kin_global.hip -- the global-memory layout, for mechanisms beyond the wave layout's 63
// species (up to 255).  The paper's first kinetics kernel (Sec. 4.2) keeps each cell's whole
// Jacobian in global memory with one thread per cell; here a cell gets a whole wavefront, and
// its matrix sits in global memory column-major, so that one column of one cell is one
// coalesced access and the wavefront's 64 lanes share each elimination step.  Every trailing
// element is read and written once per pivot step, which makes the layout bound by HBM
// bandwidth.  The matrices of a launch live in a workspace of slots, one per wavefront; a
// wavefront that finishes its cell takes the next from the work counter.
//
// Method as in the other layouts: Newton iterations on backward Euler in x = (Y, T) for a
// constant-(rho, e) cell, (I - hJ) dx = -G, dyadic sub-step halving on failure (Sec. 3.2,
// Eq. "kinetics"; energy bookkeeping of Sec. 2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kin_internal.h"

namespace kin {
namespace {

#include "kin_xlane.h"

constexpr double gTmin = 200.0, gTmax = 6000.0;

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

enum { G_CONTINUE = 0, G_ACCEPTED = 1, G_FAILED = 2 };

// ==== one wavefront per cell ======================================================================
// The cell's matrix sits in global memory column-major with column stride NP = N rounded up to
// 64, so that one column of one cell is one coalesced access of its wavefront.  Lane l owns
// rows (and unknowns) l, l + 64, l + 128, l + 192 (at most RW per lane).  Species vectors
// and the pivot row are staged in LDS; rows stay in place during the elimination (a row's
// current position is `pos`, as in the wave layout), so a step reads and writes every
// trailing element once and reads the pivot row once.

__device__ __forceinline__ int gnp(int N) { return (N + 63) & ~63; }

// element (row i, column j) of the slot's matrix
__device__ __forceinline__ double *gm(double *M, int NP, int i, int j) { return M + (size_t)j * NP + i; }

__device__ __forceinline__ double gw_sum(double v) { return wave_sum(v); }

template <int RW, typename T>
__device__ __forceinline__ T pick(const T (&v)[RW], int m)
{
    T r = v[0];
#pragma unroll
    for (int q = 1; q < RW; ++q) r = (m == q) ? v[q] : r;
    return r;
}

struct GLds {
    double *c, *g, *hh, *W, *Mc, *prow;
};

// LDS doubles per wavefront: c, g, hh (ns each), W and the pivot row (N each), the [M] slots
__host__ __device__ inline size_t glds_doubles(int ns, int ntb)
{
    return 3 * (size_t)ns + 2 * ((size_t)ns + 1) + (size_t)(ntb > 0 ? ntb : 1);
}

__device__ __forceinline__ GLds glds_map(double *p, int ns, int ntb)
{
    GLds L;
    L.c = p; p += ns;
    L.g = p; p += ns;
    L.hh = p; p += ns;
    L.W = p; p += ns + 1;
    L.prow = p; p += ns + 1;
    L.Mc = p;
    return L;
}

// Mixture e and c_v at T for the state held in x[] (lane l: unknowns l + 64 m); wave-uniform.
template <int RW>
__device__ __forceinline__ void gw_energy(const WaveTables &t, int lane, const double (&x)[RW], double T,
                                          double &e, double &cv)
{
    double es = 0.0, cs = 0.0;
    const double iT = 1.0 / T;
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int s = lane + 64 * m;
        if (s < t.ns) {
            const GThermo th = gthermo(t, s, T, iT, 0.0);
            const double rm = 8.31446261815324e3 / t.M[s];
            es = fma(x[m], rm * T * (th.h - 1.0), es);
            cs = fma(x[m], rm * (th.cp - 1.0), cs);
        }
    }
    e = gw_sum(es);
    cv = gw_sum(cs);
}

template <int RW>
__device__ bool gw_invert_T(const WaveTables &t, int lane, const double (&x)[RW], double e0, double T0,
                            double &T_out)
{
    double T = T0;
    for (int it = 0; it < 20; ++it) {
        double e, cv;
        gw_energy<RW>(t, lane, x, T, e, cv);
        if (!(cv > 0.0)) break;
        const double dT = (e - e0) / cv;
        T -= dT;
        if (!__builtin_isfinite(T) || T < gTmin || T > gTmax) break;
        if (fabs(dT) <= 1e-13 * T) { T_out = T; return true; }
    }
    double lo = gTmin, hi = gTmax, e, cv;
    gw_energy<RW>(t, lane, x, lo, e, cv);
    const double flo = e - e0;
    gw_energy<RW>(t, lane, x, hi, e, cv);
    const double fhi = e - e0;
    if (!(flo <= 0.0 && fhi >= 0.0)) return false;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * lo; ++it) {
        const double mid = 0.5 * (lo + hi);
        gw_energy<RW>(t, lane, x, mid, e, cv);
        if (e - e0 > 0.0) hi = mid; else lo = mid;
    }
    T_out = 0.5 * (lo + hi);
    return true;
}

// f (lane l: f of unknowns l + 64 m, into f[]) and the Jacobian into the slot's matrix, at xk.
template <int RW>
__device__ void gw_eval(const WaveTables &t, const GLds &L, double *Mx, int lane, double rho,
                        const double (&xk)[RW], double (&f)[RW])
{
    const int ns = t.ns, N = ns + 1, NP = gnp(N);
    const double T = rdlane(pick<RW>(xk, ns >> 6), ns & 63);
    const double iT = 1.0 / T, lT = log(T);
    const double rc = 1e-3 * rho, irc = 1.0 / rc;
    const double lPaRT = t.lnPaR - lT;
    double ek[RW], cvk[RW], dcvk[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int s = lane + 64 * m;
        ek[m] = cvk[m] = dcvk[m] = 0.0;
        if (s < ns) {
            const GThermo th = gthermo(t, s, T, iT, lT);
            const double rm = 8.31446261815324e3 / t.M[s];
            L.c[s] = xk[m] * (rc / t.M[s]);
            L.g[s] = th.h - th.s;
            L.hh[s] = th.h;
            ek[m] = rm * T * (th.h - 1.0);
            cvk[m] = rm * (th.cp - 1.0);
            dcvk[m] = rm * th.dcp;
        }
        if (s < N) L.W[s] = 0.0;
    }
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int m = 0; m < RW; ++m)
            if (lane + 64 * m < N) *gm(Mx, NP, lane + 64 * m, j) = 0.0;
    wave_sync();
    for (int q = lane; q < t.ntb; q += 64) {
        double acc = 0.0;
        for (int s = 0; s < ns; ++s) acc = fma(t.effT[(size_t)s * t.ntb + q], L.c[s], acc);
        L.Mc[q] = acc;
    }
    // the zeroing stores complete before the atomic adds
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    wave_sync();
    // reactions, one per lane; Jacobian terms by atomic adds into the slot's matrix
    const double4 *rxd4 = reinterpret_cast<const double4 *>(t.rxd);
    for (int r0 = 0; r0 < t.nr; r0 += 64) {
        const int r = r0 + lane;
        if (r >= t.nr) continue;
        const RxnRec x = t.rxc[r];
        const double4 rd = rxd4[r];
        const RxnCoef *kc = t.rxk + r;
        const double lkf = fma(-rd.z, iT, fma(rd.y, lT, rd.x));
        const double kf = exp(lkf);
        const double dlkf = fma(rd.z, iT, rd.y) * iT;
        double pw[6], dpw[6], sg = 0.0, sh = 0.0;
        int sp[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            sp[q] = x.coff[q] >> 3;
            double cq = 1.0;
            if (x.nu[q] != 0) {
                cq = L.c[sp[q]];
                sg = fma((double)x.nu[q], L.g[sp[q]], sg);
                sh = fma((double)x.nu[q], L.hh[sp[q]], sh);
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
        const double Mc = x.tb >= 0 ? L.Mc[x.tb] : 1.0;
        const double D = pf - pb;
        const double qr = Mc * D;
        const double qT = Mc * (pf * dlkf - pb * (dlkf - dlKc));
        if (x.tb >= 0) L.Mc[x.tb] = D;
#pragma unroll
        for (int k = 0; k < 6; ++k) dq[k] = Mc * dq[k] * kc->colc[k];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if (x.nu[i] == 0) continue;
            const double nu = (double)x.nu[i];
            const double a = kc->rowc[i];
            __hip_atomic_fetch_add(L.W + sp[i], nu * qr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            atomicAdd(gm(Mx, NP, sp[i], ns), nu * qT);
#pragma unroll
            for (int j = 0; j < 6; ++j)
                if (x.nu[j] != 0) atomicAdd(gm(Mx, NP, sp[i], sp[j]), a * dq[j]);
        }
    }
    // the atomic adds complete, and no stale copy of their lines stays in this CU's cache
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    wave_sync();
    // dense third-body terms, entries sorted by row: lane k sums a row's entries for its
    // columns in registers and adds each sum once
    {
        int cur = t.ntbe > 0 ? (t.tbe[0] >> 16) : 0;
        double acc[RW];
#pragma unroll
        for (int m = 0; m < RW; ++m) acc[m] = 0.0;
        for (int e = 0; e < t.ntbe; ++e) {
            const int ent = t.tbe[e];
            const int row = ent >> 16;
            if (row != cur) {
#pragma unroll
                for (int m = 0; m < RW; ++m)
                    if (lane + 64 * m < ns) { *gm(Mx, NP, cur, lane + 64 * m) += acc[m]; acc[m] = 0.0; }
                cur = row;
            }
            const double D = L.Mc[ent & 0xffff];
            const double *er = t.effR + (size_t)e * ns;
#pragma unroll
            for (int m = 0; m < RW; ++m)
                if (lane + 64 * m < ns) acc[m] = fma(D, er[lane + 64 * m], acc[m]);
        }
        if (t.ntbe > 0)
#pragma unroll
            for (int m = 0; m < RW; ++m)
                if (lane + 64 * m < ns) *gm(Mx, NP, cur, lane + 64 * m) += acc[m];
    }
    // species rows of f and the temperature column; e_s and c_v,s replace g and h
    double de = 0.0, cv = 0.0, dcv = 0.0;
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int s = lane + 64 * m;
        f[m] = 0.0;
        if (s < ns) {
            const double ms = t.M[s] * irc;
            f[m] = L.W[s] * ms;
            *gm(Mx, NP, s, ns) *= ms;
            L.g[s] = ek[m];
            L.hh[s] = cvk[m];
            de = fma(ek[m], f[m], de);
            cv = fma(xk[m], cvk[m], cv);
            dcv = fma(xk[m], dcvk[m], dcv);
        }
    }
    cv = gw_sum(cv);
    dcv = gw_sum(dcv);
    de = gw_sum(de);
    const double fT = -de / cv, icv = 1.0 / cv;
    wave_sync();
    // energy row: J[ns][k] = -(sum_s e_s J[s][k] + f_T c_v,k) / c_v, one column per step
    for (int k = 0; k <= ns; ++k) {
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int s = lane + 64 * m;
            if (s < ns) {
                part = fma(L.g[s], *gm(Mx, NP, s, k), part);
                if (k == ns) part = fma(L.hh[s], f[m], part);
            }
        }
        const double acc = gw_sum(part);
        const double v = (k < ns) ? -fma(fT, L.hh[k], acc) * icv : -fma(fT, dcv, acc) * icv;
        if (lane == 0) *gm(Mx, NP, ns, k) = v;
    }
    if ((ns & 63) == lane) f[ns >> 6] = fT;
    wave_sync();
}

// Gaussian elimination with partial pivoting over the slot's matrix, rows in place; b[] holds
// the right-hand side of the lane's rows and returns the update of its unknowns.
template <bool F32, int RW>
__device__ bool gw_solve(const GLds &L, double *Mx, int lane, int N, double (&b)[RW])
{
    using R = typename std::conditional<F32, float, double>::type;
    const int NP = gnp(N);
    int pos[RW];
    double dg[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) { pos[m] = lane + 64 * m; dg[m] = 1.0; }
    bool ok = true;
    for (int k = 0; k < N; ++k) {
        // the lane's best candidate row in column k: largest |a|, ties to the lowest position
        double v[RW];
        R best = R(-1);
        int bpos = 0x7fffffff, bm = 0;
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int i = lane + 64 * m;
            v[m] = 0.0;
            if (i < N) {
                v[m] = *gm(Mx, NP, i, k);
                const R a = (R)fabs((R)v[m]);
                if (pos[m] >= k && (a > best || (a == best && pos[m] < bpos))) { best = a; bpos = pos[m]; bm = m; }
            }
        }
        const bool cand = bpos != 0x7fffffff;
        const int w = pivot_lane<R>(cand ? best : R(0), cand, cand ? bpos : 0x7fffffff);
        const int mw = rdlane(bm, w);
        const int p = w + 64 * mw;                       // physical pivot row
        const int pos_p = rdlane(pick<RW>(pos, mw), w);
        const double piv_d = rdlane(pick<RW>(v, mw), w);
        const R piv = (R)piv_d;
        if (piv == R(0)) ok = false;
        const double yk = rdlane(pick<RW>(b, mw), w);
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int i = lane + 64 * m;
            const bool isp = i == p;
            dg[m] = isp ? piv_d : dg[m];
            pos[m] = isp ? k : (pos[m] == k ? pos_p : pos[m]);
        }
        // the pivot row's trailing part into LDS
        for (int j = k + 1 + lane; j < N; j += 64) L.prow[j] = *gm(Mx, NP, p, j);
        wave_sync();
        R l[RW];
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            l[m] = (lane + 64 * m < N && pos[m] > k) ? (R)v[m] / piv : R(0);
            b[m] = (double)fma(-l[m], (R)yk, (R)b[m]);
        }
        for (int j = k + 1; j < N; ++j) {
            const R pj = (R)L.prow[j];
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                if (l[m] != R(0)) {
                    double *e = gm(Mx, NP, lane + 64 * m, j);
                    *e = (double)fma(-l[m], pj, (R)*e);
                }
            }
        }
        wave_sync();
    }
    // back substitution by columns: the row at position k gives x_k, which every row above
    // it removes from its right-hand side
    double xl[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) xl[m] = 0.0;
    for (int k = N - 1; k >= 0; --k) {
        int o = -1, om = 0;
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const unsigned long long bal = __ballot(lane + 64 * m < N && pos[m] == k);
            if (bal) { o = __builtin_ctzll(bal); om = m; }
        }
        const double xk = (double)((R)rdlane(pick<RW>(b, om), o) / (R)rdlane(pick<RW>(dg, om), o));
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int i = lane + 64 * m;
            if (i == k) xl[m] = xk;
            if (i < N && pos[m] < k) b[m] = (double)fma(-(R)*gm(Mx, NP, i, k), (R)xk, (R)b[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < RW; ++m) b[m] = xl[m];
    return ok;
}

template <bool F32, int RW>
__global__ void __launch_bounds__(64) gwave_kernel(WaveTables t, AdvanceArgs a, double *wsbase, long long S)
{
    extern __shared__ double gsmem[];
    const long long slot = blockIdx.x;
    if (slot >= S) return;
    const int lane = threadIdx.x;
    const int ns = t.ns, N = ns + 1, NP = gnp(N);
    double *Mx = wsbase + (size_t)slot * NP * N;
    const GLds L = glds_map(gsmem, ns, t.ntb);
    const bool adapt = a.L_forced < 0;
    const int Lc = adapt ? a.L_max : a.L_forced;
    const unsigned long long end = 1ull << Lc;
    for (;;) {
        unsigned long long gi = 0;
        if (lane == 0) gi = atomicAdd(a.counter, 1ull);
        gi = __shfl(gi, 0);
        if (gi >= (unsigned long long)a.total) break;
        int j = 0;
        while (j + 1 < a.nspan && (unsigned long long)a.span[j + 1].start <= gi) ++j;
        const long long cell = (long long)gi - a.span[j].start;
        const double dt = a.span[j].dt;
        const Arena ar = arena_at(a.span[j].base, a.span[j].n, ns);
        const long long ld = a.span[j].n;
        const double rho = ar.rho[cell], e0 = ar.e0[cell];
        double x[RW], xk[RW];
        bool fin = true;
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int i = lane + 64 * m;
            x[m] = 0.0;
            if (i < ns) x[m] = ar.Y[(size_t)i * ld + cell];
            else if (i == ns) x[m] = ar.T[cell];
            xk[m] = x[m];
            fin = fin && __builtin_isfinite(x[m]);
        }
        const double T0 = ar.T[cell];
        const bool bad = __any(!fin) || !__builtin_isfinite(rho) || !(rho > 0.0) || !__builtin_isfinite(e0) ||
                         !__builtin_isfinite(dt) || !(dt >= 0.0) || T0 < gTmin || T0 > gTmax;
        if (bad) {
            if (lane == 0) {
                ar.status[cell] = 3;
                ar.level[cell] = 0;
                ar.iters[cell] = 0;
                ar.sched[cell] = 0xcbf29ce484222325ull;
            }
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
            const double h = ldexp(dt, -l);
            // one Newton iteration
            int outcome = G_CONTINUE;
            double f[RW], bv[RW];
            gw_eval<RW>(t, L, Mx, lane, rho, xk, f);
            double chk = 0.0;
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                bv[m] = 0.0;
                if (i < N) {
                    bv[m] = -((xk[m] - x[m]) - h * f[m]);
                    chk += bv[m] - bv[m];
                }
            }
            double rmax[RW];
#pragma unroll
            for (int m = 0; m < RW; ++m) rmax[m] = 0.0;
            for (int jc = 0; jc < N; ++jc)
#pragma unroll
                for (int m = 0; m < RW; ++m) {
                    const int i = lane + 64 * m;
                    if (i < N) {
                        double *e = gm(Mx, NP, i, jc);
                        const double v = (i == jc ? 1.0 : 0.0) - h * *e;
                        *e = v;
                        chk += v - v;
                        rmax[m] = fmax(rmax[m], fabs(v));
                    }
                }
            if (F32) {  // row equilibration before the FP32 factorisation
#pragma unroll
                for (int m = 0; m < RW; ++m) rmax[m] = (lane + 64 * m < N) ? 1.0 / rmax[m] : 1.0;
                for (int jc = 0; jc < N; ++jc)
#pragma unroll
                    for (int m = 0; m < RW; ++m)
                        if (lane + 64 * m < N) *gm(Mx, NP, lane + 64 * m, jc) *= rmax[m];
#pragma unroll
                for (int m = 0; m < RW; ++m) bv[m] *= rmax[m];
            }
            if (__any(!(chk == 0.0))) {
                outcome = G_FAILED;
            } else if (!gw_solve<F32, RW>(L, Mx, lane, N, bv)) {
                outcome = G_FAILED;
            } else {
                bool conv = true, finx = true;
                double r = 0.0;
#pragma unroll
                for (int m = 0; m < RW; ++m) {
                    const int i = lane + 64 * m;
                    if (i < N) {
                        xk[m] += bv[m];
                        finx = finx && __builtin_isfinite(xk[m]);
                        const double atol = (i < ns) ? a.atol_Y : a.atol_T;
                        conv = conv && (fabs(bv[m]) <= atol + a.rtol * fabs(xk[m]));
                        r = fmax(r, fabs(bv[m]) / (atol + a.rtol * fabs(xk[m])));
                    }
                }
                const double Tk = rdlane(pick<RW>(xk, ns >> 6), ns & 63);
                const bool allconv = __all(conv);
                if (__any(!finx) || Tk < gTmin || Tk > gTmax) {
                    outcome = G_FAILED;
                } else if (!allconv && !a.point_implicit) {
                    const double rw = wave_max(r);
                    if (a.diverge_ratio > 0.0 && r_prev >= 0.0 && rw > a.diverge_ratio * r_prev) outcome = G_FAILED;
                    else { if (a.diverge_ratio > 0.0) r_prev = rw; outcome = G_CONTINUE; }
                } else {
                    bool neg = false;
#pragma unroll
                    for (int m = 0; m < RW; ++m)
                        if (lane + 64 * m < ns) neg = neg || xk[m] < -a.y_neg;
                    double Tn;
                    if (!a.point_implicit && __any(neg)) {
                        outcome = G_FAILED;
                    } else if (!gw_invert_T<RW>(t, lane, xk, e0, Tk, Tn)) {
                        outcome = G_FAILED;
                    } else {
#pragma unroll
                        for (int m = 0; m < RW; ++m)
                            if (lane + 64 * m == ns) xk[m] = Tn;
                        outcome = G_ACCEPTED;
                    }
                }
            }
            if (outcome == G_CONTINUE && ++k >= a.k_max) outcome = G_FAILED;
            if (outcome == G_CONTINUE) continue;
            hsh = (hsh ^ (unsigned long long)(2 * l + (outcome == G_ACCEPTED ? 1 : 0))) * 0x100000001b3ull;
            k = 0;
            if (outcome == G_ACCEPTED) {
#pragma unroll
                for (int m = 0; m < RW; ++m) x[m] = xk[m];
                tt += 1ull << (Lc - l);
                if (adapt && l > 0 && (tt & ((1ull << (Lc - l + 1)) - 1ull)) == 0ull) --l;
                if (tt >= end) st = failed ? 1 : 0;
            } else {
#pragma unroll
                for (int m = 0; m < RW; ++m) xk[m] = x[m];
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
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                if (i < ns) ar.Y[(size_t)i * ld + cell] = x[m];
                else if (i == ns) ar.T[cell] = x[m];
            }
        }
        if (lane == 0) {
            ar.status[cell] = st;
            ar.level[cell] = level;
            ar.iters[cell] = iters;
            ar.sched[cell] = hsh;
        }
    }
}
}  // namespace

size_t global_work_doubles_per_slot(int ns, int ntb)
{
    (void)ntb;
    const size_t N = (size_t)ns + 1, NP = (N + 63) & ~(size_t)63;
    return NP * N;
}

hipError_t launch_global(const WaveTables &t, const AdvanceArgs &a, bool f32, double *work, long long slots,
                         hipStream_t s)
{
    if (slots <= 0) return hipSuccess;
    if (slots > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * glds_doubles(t.ns, t.ntb);
    if (lds > 65536) return hipErrorInvalidConfiguration;
#define KIN_GW(RWV)                                                                                  \
    case RWV:                                                                                        \
        if (f32)                                                                                     \
            hipLaunchKernelGGL((gwave_kernel<true, RWV>), dim3((unsigned)slots), dim3(64), lds, s, t, a, work, slots); \
        else                                                                                         \
            hipLaunchKernelGGL((gwave_kernel<false, RWV>), dim3((unsigned)slots), dim3(64), lds, s, t, a, work, slots); \
        break;
    switch ((t.ns + 1 + 63) / 64) {
        KIN_GW(1)
        KIN_GW(2)
        KIN_GW(3)
        KIN_GW(4)
    default:
        return hipErrorInvalidValue;
    }
#undef KIN_GW
    return hipGetLastError();
}

}  // namespace kin
