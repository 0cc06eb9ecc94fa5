// kin_global.hip -- the global-memory layout, for mechanisms beyond the wave layout's 63
// species (up to 255).  The paper's first kinetics kernel (Sec. 4.2) keeps each cell's whole
// Jacobian in global memory with one thread per cell; here a cell gets a whole wavefront, and
// its matrix sits in global memory column-major, so that one column of one cell is one
// coalesced access and the wavefront's 64 lanes share each elimination step.  The Jacobian
// is assembled by atomic adds, completed and turned into the Newton matrix in one pass over
// its columns, and factored by a blocked elimination that reads and writes each trailing
// column once per panel of pivot steps.  The matrices of a launch live in a workspace of
// slots, one per wavefront; a wavefront that finishes its cell takes the next from the work
// counter.
//
// Method as in the other layouts: Newton iterations on backward Euler in x = (Y, T) for a
// constant-(rho, e) cell, (I - hJ) dx = -G, dyadic sub-step halving on failure (Sec. 3.2,
// Eq. "kinetics"; energy bookkeeping of Sec. 2).
#include <hip/hip_runtime.h>

#include <mutex>
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
// The cell's system is padded to NQ = N rounded up to 8 unknowns with identity rows and
// columns, which leave the first N unknowns' solution unchanged and let elimination panels
// and column batches divide the system exactly.  The matrix sits in global memory
// column-major with column stride NP = NQ rounded up to 64, so that one column of one cell is
// one coalesced access of its wavefront.  Lane l owns rows (and unknowns) l, l + 64, l + 128,
// l + 192 (at most RW per lane).  Every access is unconditional (a lane with nothing to access
// in the elimination passes an out-of-range offset, see gbld), so that loads issued ahead of
// their use are not waited on early.

constexpr int kGC = 4;                                   // columns per batch

__host__ __device__ inline int gnq(int N) { return (N + 7) & ~7; }
__host__ __device__ inline int gnp(int N) { return (gnq(N) + 63) & ~63; }

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
    double *c, *g, *hh, *W, *Mc, *tq, *cb, *tgf;
    int *tgs;
};

// LDS doubles per wavefront: c, g, hh (ns each), W (N), the [M] slots (ntb), per column of a
// batch the third-body slot terms (ntb) and row sums (N), and, when `staged` entries are
// given (ntbe > 0), a copy of the slot-ordered third-body entries (factor and slot | row)
__host__ __device__ inline size_t glds_doubles(int ns, int ntb, int staged)
{
    const size_t N = (size_t)ns + 1, nb = (size_t)(ntb > 0 ? ntb : 1), ne = (size_t)(staged > 0 ? staged : 0);
    return 3 * (size_t)ns + N + nb + kGC * (nb + N) + ne + (ne + 1) / 2;
}

__device__ __forceinline__ GLds glds_map(double *p, int ns, int ntb, int ntbe)
{
    const int nb = ntb > 0 ? ntb : 1, ne = ntbe > 0 ? ntbe : 1;
    GLds L;
    L.c = p; p += ns;
    L.g = p; p += ns;
    L.hh = p; p += ns;
    L.W = p; p += ns + 1;
    L.Mc = p; p += nb;
    L.tq = p; p += kGC * nb;
    L.cb = p; p += kGC * (ns + 1);
    L.tgf = p; p += ne;
    L.tgs = reinterpret_cast<int *>(p);
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

// The Newton system at xk for a sub-step of size h: f (lane l: f of unknowns l + 64 m, into
// f[]) and the matrix I - hJ of the padded system into the slot's matrix.  rs[] returns the
// reciprocal row maxima of the lane's rows (1 for padding rows); chk accumulates v - v over
// the matrix entries (non-zero when one is not finite).
template <int RW>
__device__ void gw_system(const WaveTables &t, const GLds &L, bool staged, double *Mx, int lane, double rho,
                          double h, const double (&xk)[RW], double (&f)[RW], double (&rs)[RW], double &chk)
{
    const int ns = t.ns, N = ns + 1, NQ = gnq(N), NP = gnp(N);
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
    // the Jacobian's columns are cleared for every row a lane owns
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int m = 0; m < RW; ++m) *gm(Mx, NP, lane + 64 * m, j) = 0.0;
    for (int q = lane; q < kGC * N; q += 64) L.cb[q] = 0.0;
    wave_sync();
    // [M] of each third-body slot; four independent partial sums keep loads in flight
    for (int q = lane; q < t.ntb; q += 64) {
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        int s = 0;
        for (; s + 4 <= ns; s += 4) {
            acc0 = fma(t.effT[(size_t)s * t.ntb + q], L.c[s], acc0);
            acc1 = fma(t.effT[(size_t)(s + 1) * t.ntb + q], L.c[s + 1], acc1);
            acc2 = fma(t.effT[(size_t)(s + 2) * t.ntb + q], L.c[s + 2], acc2);
            acc3 = fma(t.effT[(size_t)(s + 3) * t.ntb + q], L.c[s + 3], acc3);
        }
        for (; s < ns; ++s) acc0 = fma(t.effT[(size_t)s * t.ntb + q], L.c[s], acc0);
        L.Mc[q] = (acc0 + acc1) + (acc2 + acc3);
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
    // species rows of f; c_v,s replaces h in LDS for the energy row
    double de = 0.0, cv = 0.0, dcv = 0.0, msr[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int s = lane + 64 * m;
        f[m] = 0.0;
        msr[m] = 0.0;
        if (s < ns) {
            msr[m] = t.M[s] * irc;
            f[m] = L.W[s] * msr[m];
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
    if ((ns & 63) == lane) f[ns >> 6] = fT;
    wave_sync();
    // One pass over the columns, kGC at a time: the dense third-body terms (slot terms of the
    // batch's columns into LDS, then one lane per entry adds into its row's LDS sum), the
    // temperature column's M_s / rho' factor, the energy row
    //   J[ns][k] = -(sum_s e_s J[s][k] + f_T c_v,k) / c_v,
    // and the Newton matrix I - hJ, padding rows and columns set to the identity.
    double rmax[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) rmax[m] = 0.0;
    for (int j = 0; j < NQ; j += kGC) {
        double a[kGC][RW];
#pragma unroll
        for (int q = 0; q < kGC; ++q)
#pragma unroll
            for (int m = 0; m < RW; ++m) a[q][m] = *gm(Mx, NP, lane + 64 * m, min(j + q, N - 1));
        if (t.ntb > 0 && j < ns) {
            // slot terms D_q eff_q,k / M_k of the batch's columns (zero past the species); a
            // batch's table loads are all issued before any is used
            for (int p0 = 0; p0 < t.ntb; p0 += 128) {
                const int pa = min(p0 + lane, t.ntb - 1), pb = min(p0 + 64 + lane, t.ntb - 1);
                double ea[kGC], eb[kGC];
#pragma unroll
                for (int q = 0; q < kGC; ++q) {
                    const size_t row0 = (size_t)min(j + q, ns - 1) * t.ntb;
                    ea[q] = t.effTM[row0 + pa];
                    eb[q] = t.effTM[row0 + pb];
                }
                const double da = L.Mc[pa], db = L.Mc[pb];
#pragma unroll
                for (int q = 0; q < kGC; ++q) {
                    const bool sp = j + q < ns;
                    if (p0 + lane < t.ntb) L.tq[q * t.ntb + pa] = sp ? da * ea[q] : 0.0;
                    if (p0 + 64 + lane < t.ntb) L.tq[q * t.ntb + pb] = sp ? db * eb[q] : 0.0;
                }
            }
            wave_sync();
            // one lane per entry adds its row's terms (entries of one slot have distinct rows)
            auto entries = [&](const int *tgs, const double *tgf) {
                for (int e = lane; e < t.ntbe; e += 64) {
                    const int ent = tgs[e];
                    const int slot = ent & 0xffff, row = ent >> 16;
                    const double fr = tgf[e];
#pragma unroll
                    for (int q = 0; q < kGC; ++q)
                        __hip_atomic_fetch_add(L.cb + q * N + row, fr * L.tq[q * t.ntb + slot], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
            };
            if (staged) entries(L.tgs, L.tgf);
            else entries(t.tgs, t.tgf);
            wave_sync();
#pragma unroll
            for (int q = 0; q < kGC; ++q)
#pragma unroll
                for (int m = 0; m < RW; ++m) {
                    const int i = lane + 64 * m;
                    if (i < ns) {
                        a[q][m] += L.cb[q * N + i];
                        L.cb[q * N + i] = 0.0;
                    }
                }
            wave_sync();
        }
        double ve[kGC];
#pragma unroll
        for (int q = 0; q < kGC; ++q) {
            const int col = j + q;
            double part = 0.0;
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int s = lane + 64 * m;
                if (s < ns) {
                    if (col == ns) a[q][m] *= msr[m];
                    part = fma(ek[m], a[q][m], part);
                    if (col == ns) part = fma(cvk[m], f[m], part);
                }
            }
            const double acc = gw_sum(part);
            const double cvc = (col < ns) ? L.hh[min(col, ns - 1)] : dcv;
            ve[q] = -fma(fT, cvc, acc) * icv;
        }
#pragma unroll
        for (int q = 0; q < kGC; ++q) {
            const int col = j + q;
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                double v;
                if (i < N && col < N) {
                    const double jv = (i == ns) ? ve[q] : a[q][m];
                    v = (i == col ? 1.0 : 0.0) - h * jv;
                    chk += v - v;
                    rmax[m] = fmax(rmax[m], fabs(v));
                } else {
                    v = (i == col && i < NQ) ? 1.0 : 0.0;
                }
                *gm(Mx, NP, i, col) = v;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < RW; ++m) rs[m] = (lane + 64 * m < N) ? 1.0 / rmax[m] : 1.0;
}

// The elimination addresses the slot's matrix through a buffer resource: one scalar base,
// a scalar column offset and a 32-bit lane (row) offset per access, so a batch of column
// accesses shares one address register.  A lane with nothing to access gives an offset past
// the slot (kNoRow): the hardware's range check drops its store and returns zero to its load.
typedef unsigned int gu2 __attribute__((ext_vector_type(2)));
constexpr unsigned kNoRow = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t gslot_rsrc(double *Mx, int NP, int NQ)
{
    return __builtin_amdgcn_make_buffer_rsrc(Mx, (short)0, NP * NQ * (int)sizeof(double), 0x00020000);
}

__device__ __forceinline__ double gbld(__amdgpu_buffer_rsrc_t r, unsigned row_off, int col_off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, row_off, col_off, 0));
}

__device__ __forceinline__ void gbst(__amdgpu_buffer_rsrc_t r, unsigned row_off, int col_off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(gu2, v), r, row_off, col_off, 0);
}

// Load of an element as the factorisation's type, scaled by the row factor sc (FP32 form,
// first panel only).
template <bool F32>
__device__ __forceinline__ typename std::conditional<F32, float, double>::type gld(double v, double sc)
{
    if constexpr (F32) return (float)(v * sc);
    else return v;
}

// Exchange rows k and p (physical rows of the lane-distributed vector v: lane r & 63,
// register r >> 6); wave-uniform k and p.
template <int RW, typename T>
__device__ __forceinline__ void gswap(T (&v)[RW], int lane, int k, int p)
{
    const T vk = rdlane(pick<RW>(v, k >> 6), k & 63);
    const T vp = rdlane(pick<RW>(v, p >> 6), p & 63);
#pragma unroll
    for (int m = 0; m < RW; ++m) {
        const int i = lane + 64 * m;
        v[m] = i == k ? vp : (i == p ? vk : v[m]);
    }
}

// Gaussian elimination with partial pivoting over the padded system in the slot's matrix;
// b[] holds the right-hand side of the lane's rows (already scaled by rs[] in the FP32 form,
// whose matrix rows are scaled by rs[] as the first panel reads them) and returns the update
// of its unknowns.
//
// Blocked right-looking form with physical row exchanges: a panel of GB columns is loaded
// into registers and factored there (pivot search over the rows not yet pivoted, exchange of
// the pivot row into place, multipliers, updates of the panel's later columns by readlane
// broadcasts of the pivot row), its multipliers kept in the final row order as later
// exchanges happen.  The columns right of the panel then receive the panel's exchanges and
// its GB updates in one pass, each column read and written once per panel instead of once per
// pivot step; this is the arithmetic of the unblocked order.  Rows not yet pivoted stay
// contiguous (rows k0 and up), so a panel touches whole lines of them only; lanes with
// nothing to load or store pass an out-of-range offset.  Columns move in batches (eight when
// a lane holds at most two rows, else four) with the next batch's loads issued before the
// current batch is computed.
template <bool F32, int RW>
__device__ bool gw_solve(double *Mx, int lane, int N, const double (&rs)[RW], double (&b)[RW])
{
    using R = typename std::conditional<F32, float, double>::type;
    constexpr int GB = RW <= 2 ? 8 : 4;                  // panel width (divides NQ)
    constexpr int GC = GB;                               // trailing columns per batch
    constexpr int GK = kGC;                              // back-substitution columns per batch
    const int NQ = gnq(N), NP = gnp(N), CB = NP * (int)sizeof(double);
    const __amdgpu_buffer_rsrc_t mr = gslot_rsrc(Mx, NP, NQ);
    __asm__ volatile("" ::: "memory");                   // the column pass's stores come first
    double dg[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) dg[m] = 1.0;
    bool ok = true;
    for (int k0 = 0; k0 < NQ; k0 += GB) {
        // rows k0.. are not yet pivoted: the only rows this panel changes
        unsigned ri[RW], rp[RW];
        double sc[RW];
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int i = lane + 64 * m;
            ri[m] = (i >= k0 && i < NQ) ? (unsigned)i * 8u : kNoRow;
            rp[m] = (i >= k0 && i < k0 + GB) ? (unsigned)i * 8u : kNoRow;  // the panel's own rows
            sc[m] = (k0 == 0) ? rs[m] : 1.0;
        }
        R P[GB][RW];
#pragma unroll
        for (int c = 0; c < GB; ++c)
#pragma unroll
            for (int m = 0; m < RW; ++m) P[c][m] = gld<F32>(gbld(mr, ri[m], (k0 + c) * CB), sc[m]);
        R Lp[GB][RW];
        int pv[GB];
#pragma unroll
        for (int c = 0; c < GB; ++c) {
            const int k = k0 + c;
            // the lane's best candidate row in column k: largest |a|, ties to the lowest row
            R best = R(-1);
            int bpos = 0x7fffffff;
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                const R av = (R)fabs(P[c][m]);
                if (i >= k && i < NQ && (av > best || (av == best && i < bpos))) { best = av; bpos = i; }
            }
            const bool cand = bpos != 0x7fffffff;
            const int w = pivot_lane<R>(cand ? best : R(0), cand, cand ? bpos : 0x7fffffff);
            const int p = rdlane(bpos, w);               // physical pivot row, >= k
            pv[c] = p;
            if (p != k) {                                // exchange rows k and p
#pragma unroll
                for (int c2 = c; c2 < GB; ++c2) gswap<RW>(P[c2], lane, k, p);
#pragma unroll
                for (int c1 = 0; c1 < c; ++c1) gswap<RW>(Lp[c1], lane, k, p);
                gswap<RW>(b, lane, k, p);
            }
            const R piv = rdlane(pick<RW>(P[c], k >> 6), k & 63);
            if (piv == R(0)) ok = false;
            const double yk = rdlane(pick<RW>(b, k >> 6), k & 63);
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                dg[m] = i == k ? (double)piv : dg[m];
                Lp[c][m] = (i > k && i < NQ) ? P[c][m] / piv : R(0);
                b[m] = (double)fma(-Lp[c][m], (R)yk, (R)b[m]);
            }
#pragma unroll
            for (int c2 = c + 1; c2 < GB; ++c2) {
                const R u = rdlane(pick<RW>(P[c2], k >> 6), k & 63);
#pragma unroll
                for (int m = 0; m < RW; ++m) P[c2][m] = fma(-Lp[c][m], u, P[c2][m]);
            }
        }
        // the panel's rows back (their U entries); the multipliers are not stored
#pragma unroll
        for (int c = 0; c < GB; ++c)
#pragma unroll
            for (int m = 0; m < RW; ++m) gbst(mr, rp[m], (k0 + c) * CB, (double)P[c][m]);
        // columns right of the panel: the panel's exchanges, then its GB updates per column
        const int j0 = k0 + GB;
        R nx[GC][RW];
#pragma unroll
        for (int q = 0; q < GC; ++q)
#pragma unroll
            for (int m = 0; m < RW; ++m) nx[q][m] = gld<F32>(gbld(mr, ri[m], min(j0 + q, NQ - 1) * CB), sc[m]);
        for (int j = j0; j < NQ; j += GC) {
            R cu[GC][RW];
#pragma unroll
            for (int q = 0; q < GC; ++q)
#pragma unroll
                for (int m = 0; m < RW; ++m) cu[q][m] = nx[q][m];
#pragma unroll
            for (int q = 0; q < GC; ++q)
#pragma unroll
                for (int m = 0; m < RW; ++m)
                    nx[q][m] = gld<F32>(gbld(mr, ri[m], min(j + GC + q, NQ - 1) * CB), sc[m]);
#pragma unroll
            for (int c = 0; c < GB; ++c)
                if (pv[c] != k0 + c)
#pragma unroll
                    for (int q = 0; q < GC; ++q) gswap<RW>(cu[q], lane, k0 + c, pv[c]);
#pragma unroll
            for (int c = 0; c < GB; ++c) {
                const int k = k0 + c;
#pragma unroll
                for (int q = 0; q < GC; ++q) {
                    const R u = rdlane(pick<RW>(cu[q], k >> 6), k & 63);
#pragma unroll
                    for (int m = 0; m < RW; ++m) cu[q][m] = fma(-Lp[c][m], u, cu[q][m]);
                }
            }
#pragma unroll
            for (int q = 0; q < GC; ++q)
#pragma unroll
                for (int m = 0; m < RW; ++m) gbst(mr, ri[m], (j + q) * CB, (double)cu[q][m]);
        }
    }
    // back substitution by columns over the first N rows (the padding unknowns are zero):
    // row k gives x_k, which every row above it removes from its right-hand side; a batch's
    // column entries (rows above the diagonal) are loaded one batch ahead
    double xl[RW];
#pragma unroll
    for (int m = 0; m < RW; ++m) xl[m] = 0.0;
    R ux[GK][RW];
#pragma unroll
    for (int q = 0; q < GK; ++q)
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int k = N - 1 - q, i = lane + 64 * m;
            const bool need = i < k;
            ux[q][m] = (R)gbld(mr, need ? (unsigned)i * 8u : kNoRow, max(k, 0) * CB);
        }
    for (int kt = N - 1; kt >= 0; kt -= GK) {
        R uc[GK][RW];
#pragma unroll
        for (int q = 0; q < GK; ++q)
#pragma unroll
            for (int m = 0; m < RW; ++m) uc[q][m] = ux[q][m];
#pragma unroll
        for (int q = 0; q < GK; ++q)
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int k = kt - GK - q, i = lane + 64 * m;
                const bool need = i < k;
                ux[q][m] = (R)gbld(mr, need ? (unsigned)i * 8u : kNoRow, max(k, 0) * CB);
            }
#pragma unroll
        for (int q = 0; q < GK; ++q) {
            const int k = kt - q;
            if (k < 0) continue;
            const double xk = (double)((R)rdlane(pick<RW>(b, k >> 6), k & 63) / (R)rdlane(pick<RW>(dg, k >> 6), k & 63));
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                if (i == k) xl[m] = xk;
                if (i < k) b[m] = (double)fma(-uc[q][m], (R)xk, (R)b[m]);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < RW; ++m) b[m] = xl[m];
    __asm__ volatile("" ::: "memory");                   // before the next evaluation's stores
    return ok;
}

template <bool F32, int RW>
__global__ void __launch_bounds__(64) gwave_kernel(WaveTables t, AdvanceArgs a, double *wsbase, long long S,
                                                   int staged)
{
    extern __shared__ double gsmem[];
    const long long slot = blockIdx.x;
    if (slot >= S) return;
    const int lane = threadIdx.x;
    const int ns = t.ns, N = ns + 1, NP = gnp(N);
    double *Mx = wsbase + (size_t)slot * NP * gnq(N);
    const GLds L = glds_map(gsmem, ns, t.ntb, staged ? t.ntbe : 0);
    // the slot-ordered third-body entries, read once per column batch, stay in LDS when they fit
    if (staged) {
        for (int e = lane; e < t.ntbe; e += 64) {
            L.tgs[e] = t.tgs[e];
            L.tgf[e] = t.tgf[e];
        }
    }
    wave_sync();
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
        const long long pos = (long long)gi - a.span[j].start;
        long long cell = pos;
        if (a.span[j].order) {
            const long long c = a.span[j].order[pos];
            if ((unsigned long long)c < (unsigned long long)a.span[j].n) cell = c;
        }
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
        ScheduleTrace tr;
        tr.start(a.trace, a.trace_words, a.span[j].start + cell);
        const bool bad = __any(!fin) || !__builtin_isfinite(rho) || !(rho > 0.0) || !__builtin_isfinite(e0) ||
                         !__builtin_isfinite(dt) || !(dt >= 0.0) || T0 < gTmin || T0 > gTmax;
        if (bad) {
            if (lane == 0) {
                ar.status[cell] = 3;
                ar.level[cell] = 0;
                ar.iters[cell] = 0;
                ar.sched[cell] = 0xcbf29ce484222325ull;
            }
            tr.finish(lane);
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
            double chk = 0.0, rs[RW];
            gw_system<RW>(t, L, staged != 0, Mx, lane, rho, h, xk, f, rs, chk);
#pragma unroll
            for (int m = 0; m < RW; ++m) {
                const int i = lane + 64 * m;
                bv[m] = 0.0;
                if (i < N) {
                    bv[m] = -((xk[m] - x[m]) - h * f[m]);
                    chk += bv[m] - bv[m];
                    if (F32) bv[m] *= rs[m];   // row equilibration of the FP32 factorisation
                }
            }
            if (__any(!(chk == 0.0))) {
                outcome = G_FAILED;
            } else if (!gw_solve<F32, RW>(Mx, lane, N, rs, bv)) {
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
            tr.add(outcome == G_ACCEPTED, lane);
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
        tr.finish(lane);
    }
}
}  // namespace

// Fixed device memory of the allocation-free advance (kin_advance_noalloc): its work counters
// and the matrices of its global-layout launches, in place of the counters and the
// stream-ordered workspace that kin_advance allocates.  Every device the library runs on holds
// its own copy until the process ends.  Host code never uses this name as an address: the
// per-device address comes from scratch_address().
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *addr[kScratchMaxDevices] = {};
    if (device < 0 || device >= kScratchMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *p = nullptr;
        // the caller has made `device` current
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<unsigned char *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

size_t global_work_doubles_per_slot(int ns, int ntb)
{
    (void)ntb;
    return (size_t)gnp(ns + 1) * (size_t)gnq(ns + 1);
}

hipError_t launch_global(const WaveTables &t, const AdvanceArgs &a, bool f32, double *work, long long slots,
                         hipStream_t s)
{
    if (slots <= 0) return hipSuccess;
    if (slots > 0x7fffffffLL) return hipErrorInvalidValue;
    // the third-body entries are staged in LDS when they fit in the 64 KiB of a workgroup
    int staged = t.ntbe;
    size_t lds = sizeof(double) * glds_doubles(t.ns, t.ntb, staged);
    if (lds > 65536) {
        staged = 0;
        lds = sizeof(double) * glds_doubles(t.ns, t.ntb, 0);
    }
    if (lds > 65536) return hipErrorInvalidConfiguration;
#define KIN_GW(RWV)                                                                                  \
    case RWV:                                                                                        \
        if (f32)                                                                                     \
            hipLaunchKernelGGL((gwave_kernel<true, RWV>), dim3((unsigned)slots), dim3(64), lds, s, t, a, work, slots, staged); \
        else                                                                                         \
            hipLaunchKernelGGL((gwave_kernel<false, RWV>), dim3((unsigned)slots), dim3(64), lds, s, t, a, work, slots, staged); \
        break;
    switch ((gnq(t.ns + 1) + 63) / 64) {
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
