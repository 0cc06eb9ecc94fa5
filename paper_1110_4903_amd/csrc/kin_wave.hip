// kin_wave.hip -- table-driven kernels: the wave layout (one cell per 64-wide wavefront) and
// the initial-energy kernel.
//
// Method (Le & Cambier, arXiv:1110.4903): rates from the Arrhenius law, reverse rates from
// the equilibrium constant and third-body sums (Sec. 3.2); the point-implicit system
// (I - h dOmega/dQ) dQ = -G (Sec. 3.2, Eq. "kinetics") iterated as Newton's method on
// backward Euler; Gaussian elimination with partial pivoting per cell (Sec. 4.2).  The paper
// stored a cell's Jacobian either in global memory or in one thread block's shared memory;
// here a cell owns one wavefront:
//   * lanes evaluate reactions 64 at a time and add each reaction's terms straight into the
//     cell's Jacobian in LDS with LDS atomic adds (no per-row gather lists); the dense
//     third-body terms go in afterwards as a small matrix product on the FP64 matrix cores;
//   * FP64: the augmented Newton matrix is formed in place of J in LDS and eliminated there,
//     blocked by four columns: panel pivot steps with one row (or column) per lane and
//     physical row exchanges, then the trailing update as 16 x 16 tiles on the FP64 matrix
//     instructions; back substitution with one row per lane;
//   * FP32-LU: each lane holds one row of the FP32 Newton matrix in registers; the elimination
//     runs as a loop over blocks of four pivot steps (the row is rotated by four registers
//     after each block, so every step addresses its pivot column at a compile-time register)
//     and the pivot row reaches the other lanes by readlane.
// Both pivot searches are a DPP butterfly inside 16-lane rows plus a read of the four row
// winners.
// Wavefronts never synchronise with each other, so cells with different iteration counts do
// not wait for one another.
#include <hip/hip_runtime.h>

#include "kin_internal.h"

namespace kin {

namespace {

#include "kin_xlane.h"

// NASA-7 functions of species s at T from the table.
struct Thermo {
    double cp, h, s, dcp;
};

__device__ __forceinline__ Thermo thermo(const WaveTables &t, int s, double T, double iT, double lT)
{
    const double *a = t.nasa + 14 * s + (T < t.Tmid[s] ? 0 : 7);
    Thermo o;
    o.cp = fma(T, fma(T, fma(T, fma(T, a[4], a[3]), a[2]), a[1]), a[0]);
    o.h = fma(a[5], iT, fma(T, fma(T, fma(T, fma(T, a[4] * 0.2, a[3] * 0.25), a[2] * (1.0 / 3.0)), a[1] * 0.5), a[0]));
    o.s = fma(a[0], lT, fma(T, fma(T, fma(T, fma(T, a[4] * 0.25, a[3] * (1.0 / 3.0)), a[2] * 0.5), a[1]), a[6]));
    o.dcp = fma(T, fma(T, fma(T, 4.0 * a[4], 3.0 * a[3]), 2.0 * a[2]), a[1]);
    return o;
}

// ---- per-wavefront LDS layout (in doubles) --------------------------------------------------
// [0, R)            J[N][NPAD + 1] (columns N.. stay zero), then the FP64 Newton matrix
//                   [I - hJ | b] in place; the odd row stride lets a column read by one lane
//                   per row hit distinct banks
//                   (the last row stops after column N)
// W[N + 1]          net production sums, then f (the T-derivative sums accumulate straight
//                   into J's column N - 1 and are scaled there)
// c, g, hh          concentrations, g/RT and h/RT for the rates, then e_s and cv_s for the
//                   energy row: when N <= NPAD - 3 ("packed") they are the columns JS - 1, JS - 2
//                   and JS - 3 of J's species rows, which the matrix never uses; otherwise three
//                   vectors of N entries after W
// Mc[ntb]           third-body concentrations; each is replaced by its reaction's q_f - q_b
//                   (one reaction per slot reads, then writes, its own entry)
// 12.8 KB for the 36-species mechanism (packed), which leaves room for twelve wavefronts on a
// compute unit
__host__ __device__ inline int round_even(int x) { return (x + 1) & ~1; }

// row stride of J and the Newton matrix, in entries of 8 bytes
__host__ __device__ constexpr int j_stride(int npad) { return npad + 1; }

__host__ __device__ inline int j_entries(int N, int npad) { return (N - 1) * j_stride(npad) + N + 1; }

__host__ __device__ inline int j_region(int N, int npad) { return round_even(j_entries(N, npad)); }

// the species vectors fit in J's unused columns
__host__ __device__ constexpr bool packed_vectors(int N, int npad) { return N <= npad - 3; }

__host__ __device__ inline size_t lds_doubles(int N, int ntb, int npad)
{
    const size_t vec = packed_vectors(N, npad) ? 0 : 3 * (size_t)round_even(N);
    return (size_t)j_region(N, npad) + (size_t)round_even(N + 1) + vec + (size_t)round_even(ntb);
}

struct Lds {
    double *J, *W, *c, *g, *hh, *Mc;
};

typedef double dvec4 __attribute__((ext_vector_type(4)));

template <bool PK>
__device__ __forceinline__ Lds lds_map(double *base, int N, int npad)
{
    Lds L;
    double *p = base;
    L.J = p; p += j_region(N, npad);
    L.W = p; p += round_even(N + 1);
    if (PK) {
        L.c = L.J + (j_stride(npad) - 1);
        L.g = L.J + (j_stride(npad) - 2);
        L.hh = L.J + (j_stride(npad) - 3);
    } else {
        L.c = p; p += round_even(N);
        L.g = p; p += round_even(N);
        L.hh = p; p += round_even(N);
    }
    L.Mc = p;
    return L;
}

__device__ __forceinline__ void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Mixture e and c_v at T (wave-wide sums).  Every lane returns the same values.
__device__ __forceinline__ void mix_energy(const WaveTables &t, int lane, double xs, double T,
                                           double &e, double &cv)
{
    double es = 0.0, cs = 0.0;
    if (lane < t.ns) {
        const Thermo th = thermo(t, lane, T, 1.0 / T, 0.0);
        const double rm = 8.31446261815324e3 / t.M[lane];
        es = xs * (rm * T * (th.h - 1.0));
        cs = xs * (rm * (th.cp - 1.0));
    }
    e = wave_sum(es);
    cv = wave_sum(cs);
}

__device__ __forceinline__ bool invert_T(const WaveTables &t, int lane, double xs, double e0,
                                         double T0, double &T_out)
{
    double T = T0;
    for (int it = 0; it < 20; ++it) {
        double e, cv;
        mix_energy(t, lane, xs, T, e, cv);
        if (!(cv > 0.0)) break;
        const double dT = (e - e0) / cv;
        T -= dT;
        if (!__builtin_isfinite(T) || T < kTmin || T > kTmax) break;
        if (fabs(dT) <= 1e-13 * T) { T_out = T; return true; }
    }
    double lo = kTmin, hi = kTmax, e, cv;
    mix_energy(t, lane, xs, lo, e, cv);
    const double flo = e - e0;
    mix_energy(t, lane, xs, hi, e, cv);
    const double fhi = e - e0;
    if (!(flo <= 0.0 && fhi >= 0.0)) return false;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * lo; ++it) {
        const double mid = 0.5 * (lo + hi);
        mix_energy(t, lane, xs, mid, e, cv);
        if (e - e0 > 0.0) hi = mid; else lo = mid;
    }
    T_out = 0.5 * (lo + hi);
    return true;
}

// c^nu and d(c^nu)/dc = nu c^(nu-1) for nu in 0..3, without branches: h = c^(nu-1) (1 for
// nu <= 1) is a product of selected factors, then c^nu = (nu >= 1 ? c : 1) h.
__device__ __forceinline__ void cpow_nu(double c, int nu, double &p, double &dp)
{
    const double h = (nu >= 2 ? c : 1.0) * (nu >= 3 ? c : 1.0);
    p = (nu >= 1 ? c : 1.0) * h;
    dp = (double)nu * h;
}

// Rates and Jacobian terms of reaction r (lane-owned), added into W and J.
//   Q_r = [M]_r (k_f prod c^nu' - k_b prod c^nu''),  dQ_r/dc over the six species slots,
//   J[s][k] += (nu_s M_s)(dQ_r/dc_k / M_k),  W[s] += nu_s Q_r,  J[s][N-1] += nu_s dQ_r/dT.
// Slots 0-2 are the reactants, 3-5 the products; a species on both sides appears in one slot
// of each, and its two terms add up in J.  The loops over slots stop at the pass's largest
// counts (rmax reactants, pmax products); shorter reactions' unused slots add exact zeros.
// RM, PM > 0 fix those counts at compile time (the two-reactant, two-product passes that most
// reactions fall into), which turns the slot tests into constants.
template <int NPAD, int RM, int PM, bool PK>
__device__ __forceinline__ void reaction_terms(const WaveTables &t, const Lds &L, int r, const RxnRec &x,
                                               const double4 &rd, int rmax, int pmax, double iT,
                                               double lT, double lPaRT)
{
    const double lnA = rd.x, b = rd.y, Ta = rd.z, dnu = rd.w;
    const RxnCoef *kc = t.rxk + r;
    const char *cb = reinterpret_cast<const char *>(L.c);
    const char *gb = reinterpret_cast<const char *>(L.g);
    const char *hb = reinterpret_cast<const char *>(L.hh);
    const auto used = [&](int q) {
        return q < 3 ? q < (RM > 0 ? RM : rmax) : q - 3 < (PM > 0 ? PM : pmax);
    };
    const double lkf = fma(-Ta, iT, fma(b, lT, lnA));
    const double kf = exp(lkf);
    const double dlkf = fma(Ta, iT, b) * iT;
    // slot concentrations, their powers c^|nu| and derivatives, and the equilibrium sums
    double pw[6], dpw[6], gv[6], hv[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double c = 1.0;
        gv[q] = 0.0;
        hv[q] = 0.0;
        if (used(q)) {
            // packed species vectors sit one per Jacobian row: the row offset addresses them
            const int vo = PK ? x.roff[q] : x.coff[q];
            c = *reinterpret_cast<const double *>(cb + vo);
            gv[q] = *reinterpret_cast<const double *>(gb + vo);
            hv[q] = *reinterpret_cast<const double *>(hb + vo);
        }
        cpow_nu(c, q < 3 ? -x.nu[q] : x.nu[q], pw[q], dpw[q]);
    }
    const double pf = kf * (pw[0] * pw[1] * pw[2]);
    double dq[6];
    dq[0] = kf * (dpw[0] * pw[1] * pw[2]);
    dq[1] = kf * (pw[0] * dpw[1] * pw[2]);
    dq[2] = kf * (pw[0] * pw[1] * dpw[2]);
    double sg = 0.0, sh = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (used(q)) {
            const double nu = (double)x.nu[q];
            sg = fma(nu, gv[q], sg);
            sh = fma(nu, hv[q], sh);
        }
    }
    const double lKc = dnu * lPaRT - sg;
    const double kb = exp(lkf - lKc);
    const double dlKc = (sh - dnu) * iT;
    // irreversible reactions take k_b = 0 by selection (k_b itself may overflow)
    const bool rev = x.rev != 0;
    const double pb = rev ? kb * (pw[3] * pw[4] * pw[5]) : 0.0;
    dq[3] = rev ? -kb * (dpw[3] * pw[4] * pw[5]) : 0.0;
    dq[4] = rev ? -kb * (pw[3] * dpw[4] * pw[5]) : 0.0;
    dq[5] = rev ? -kb * (pw[3] * pw[4] * dpw[5]) : 0.0;
    const double Mc_read = (t.ntb > 0) ? L.Mc[x.tb >= 0 ? x.tb : 0] : 1.0;  // read on every lane
    const double Mc = (x.tb >= 0) ? Mc_read : 1.0;
    const double D = pf - pb;
    const double q = Mc * D;
    const double qT = Mc * (pf * dlkf - pb * (dlkf - dlKc));
    if (x.tb >= 0) L.Mc[x.tb] = D;  // the slot's [M] has been read; the dense pass needs D
#pragma unroll
    for (int k = 0; k < 6; ++k) dq[k] = Mc * dq[k] * kc->colc[k];  // dQ/dc_k / M_k
    char *Jb = reinterpret_cast<char *>(L.J);
    char *Wb = reinterpret_cast<char *>(L.W);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (used(i)) {
            const double nu = (double)x.nu[i];
            const double a = kc->rowc[i];
            lds_add(reinterpret_cast<double *>(Wb + x.coff[i]), nu * q);
            char *Jr = Jb + x.roff[i];
            lds_add(reinterpret_cast<double *>(Jr + 8 * t.ns), nu * qT);
#pragma unroll
            for (int j = 0; j < 6; ++j)
                if (used(j)) lds_add(reinterpret_cast<double *>(Jr + x.coff[j]), a * dq[j]);
        }
    }
}

// f = dx/dt and J = df/dx of the cell at x (lane i holds x_i).  Leaves J in L.J (row-major,
// stride NPAD, zero beyond column N - 1) and f in L.W.
template <int NPAD, bool PK>
__device__ __forceinline__ void eval(const WaveTables &t, const Lds &L, int lane, double rho, double xs,
                                     double Ms, double invMs)
{
    const int ns = t.ns, N = ns + 1, JS = j_stride(NPAD);
    constexpr int VS = PK ? j_stride(NPAD) : 1;  // stride of the species vectors
    const double T = rdlane(xs, ns);
    const double iT = 1.0 / T, lT = log(T);
    const double rc = 1e-3 * rho, irc = 1.0 / rc;
    const double lPaRT = t.lnPaR - lT;  // ln(P_atm / (R T)), CGS
    {   // clear J and W (J's region ends where W begins)
        double2 *z = reinterpret_cast<double2 *>(L.J);
        const int nj = j_entries(N, NPAD) / 2, n2 = nj + round_even(N + 1) / 2;
        const int skip = j_region(N, NPAD) / 2 - nj;
        for (int k = lane; k < n2; k += kW) z[k < nj ? k : k + skip] = make_double2(0.0, 0.0);
    }
    double cvk = 0.0, dcvk = 0.0, ek = 0.0;
    if (lane < ns) {
        const Thermo th = thermo(t, lane, T, iT, lT);
        const double rm = 8.31446261815324e3 * invMs;
        L.c[lane * VS] = xs * (rc * invMs);
        L.g[lane * VS] = th.h - th.s;
        L.hh[lane * VS] = th.h;
        ek = rm * T * (th.h - 1.0);
        cvk = rm * (th.cp - 1.0);
        dcvk = rm * th.dcp;
    }
    wave_sync();
    // third-body concentrations [M]_r = sum_s eff_rs c_s, one reaction per lane
    for (int r = lane; r < t.ntb; r += kW) {
        double acc = 0.0;
        const double *e = t.effT + r;
#pragma unroll 4
        for (int s = 0; s < ns; ++s, e += t.ntb) acc = fma(*e, L.c[s * VS], acc);
        L.Mc[r] = acc;
    }
    wave_sync();
    {   // reactions, 64 at a time; each pass loads the next pass's records
        const double4 *rxd4 = reinterpret_cast<const double4 *>(t.rxd);
        RxnRec xn{};
        double4 rn{};
        if (lane < t.nr) { xn = t.rxc[lane]; rn = rxd4[lane]; }
        for (int r0 = 0; r0 < t.nr; r0 += kW) {
            const int r = r0 + lane;
            const RxnRec x = xn;
            const double4 rd = rn;
            const int rp = uniform_table(t.chunk_rp)[r0 / kW];
            if (r + kW < t.nr) { xn = t.rxc[r + kW]; rn = rxd4[r + kW]; }
            if (r < t.nr) {
                if (rp == (2 | 2 << 8))
                    reaction_terms<NPAD, 2, 2, PK>(t, L, r, x, rd, 2, 2, iT, lT, lPaRT);
                else
                    reaction_terms<NPAD, 0, 0, PK>(t, L, r, x, rd, rp & 0xff, rp >> 8, iT, lT, lPaRT);
            }
        }
    }
    wave_sync();
    // dense third-body terms: J[s][k] gains sum_q (nu_qs M_s D_q)(eff_qk / M_k) over the
    // third-body slots q (D_q = q_f - q_b), a product of an ns x ntb and an ntb x ns matrix
    // that the FP64 matrix instruction forms in 16 x 16 output tiles, four slots per step.  The
    // host stores both factors' constant parts in the instruction's operand order, padded to
    // NT = NPAD / 16 (rounded up) row tiles and to whole batches of four steps, so each operand
    // is one coalesced load and a batch's loads are all in flight together; the left operand
    // is scaled by D_q of the lane's slot
    if (t.ntb > 0) {
        constexpr int NT = (NPAD + 15) / 16;
        const int nb = (t.ntb + 15) / 16;
        const int g = lane >> 4, c16 = lane & 15;
#pragma unroll 1
        for (int ti = 0; ti < NT; ++ti) {
            dvec4 acc[NT];
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) acc[tj] = dvec4{0.0, 0.0, 0.0, 0.0};
            const double *pa = t.tbA + (size_t)ti * 64 + lane;
            const double *pb = t.tbB + lane;
            // the last row tile needs only the slots numbered first (those with a participant in
            // its rows): its product stops after their batches
            const int nbt = ti == NT - 1 ? (t.tb_last + 15) / 16 : nb;
#pragma unroll 1
            for (int bt = 0; bt < nbt; ++bt) {
                double av[4], dv[4], bv[4][NT];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const size_t kk = 4 * bt + u;
                    av[u] = pa[kk * NT * 64];
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj) bv[u][tj] = pb[(kk * NT + tj) * 64];
                    const int q = 4 * (int)kk + g;
                    dv[u] = L.Mc[q < t.ntb ? q : t.ntb - 1];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double a = av[u] * (4 * (4 * bt + u) + g < t.ntb ? dv[u] : 0.0);
#pragma unroll
                    for (int tj = 0; tj < NT; ++tj)
                        acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[u][tj], acc[tj], 0, 0, 0);
                }
            }
            // accumulator register r of lane l is output row 4 r + l / 16, column l % 16.  Rows
            // and columns past the species are exact zeros; the adds that would fall outside the
            // species block go to the energy row instead, which is assigned afterwards
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) {
                const int k = 16 * tj + c16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int srow = 16 * ti + 4 * r + g;
                    const bool in = srow < ns && k < ns;
                    lds_add(L.J + (in ? (size_t)srow * JS + k : (size_t)ns * JS + c16), in ? acc[tj][r] : 0.0);
                }
            }
        }
    }
    wave_sync();
    // species rows of f and the temperature column; e_s and cv_s replace g and h
    double fs = 0.0;
    if (lane < ns) {
        const double ms = Ms * irc;
        fs = L.W[lane] * ms;
        L.J[(size_t)lane * JS + ns] *= ms;
        L.W[lane] = fs;
        L.g[lane * VS] = ek;
        L.hh[lane * VS] = cvk;
    }
    const double cv = wave_sum(lane < ns ? xs * cvk : 0.0);
    const double dcv = wave_sum(lane < ns ? xs * dcvk : 0.0);
    const double de = wave_sum(ek * fs);
    const double fT = -de / cv;
    const double icv = 1.0 / cv;
    wave_sync();
    // energy row: lane k < ns forms J[ns][k]; lane ns forms J[ns][ns]
    const double *E = L.g, *CV = L.hh;
    if (lane <= ns) {
        double acc = 0.0;
        if (lane < ns) {
#pragma unroll 4
            for (int s = 0; s < ns; ++s) acc = fma(E[s * VS], L.J[(size_t)s * JS + lane], acc);
            L.J[(size_t)ns * JS + lane] = -fma(fT, cvk, acc) * icv;
        } else {
#pragma unroll 4
            for (int s = 0; s < ns; ++s) acc = fma(CV[s * VS], L.W[s], fma(E[s * VS], L.J[(size_t)s * JS + ns], acc));
            L.J[(size_t)ns * JS + ns] = -fma(fT, dcv, acc) * icv;
            L.W[ns] = fT;
        }
    }
    wave_sync();
}

// The register elimination's multipliers are a_ik times this reciprocal of the pivot: in FP32
// the hardware reciprocal refined by one Newton step (within an ulp), in FP64 the quotient
template <typename R>
__device__ __forceinline__ R rpiv_of(R p)
{
    if constexpr (sizeof(R) == 4) {
        const float y = __builtin_amdgcn_rcpf(p);
        return fmaf(y, fmaf(-p, y, 1.0f), y);
    } else {
        return R(1) / p;
    }
}

// Gaussian elimination with partial pivoting, one row per lane, and back substitution.  Lane
// i < N enters with row i of A in a[] and b_i in bb; on return x holds solution component
// `lane` (lanes >= N: 0).  Pivot rule: the row of largest |a_ik| among rows not yet used,
// ties to the lowest current position.  Rows never move between lanes: `pos` is the row's
// current position, and the lane that supplies pivot k keeps its row, now row k of U, frozen
// in its registers, where the back substitution reads it.  The pivot row reaches the other
// lanes by readlane.  Returns false on an exactly zero pivot.
template <int NPAD, typename R>
__device__ __forceinline__ bool lu_solve(R (&a)[NPAD], R bb, int N, int lane, R &x)
{
    constexpr int B = kLuBlock;
    static_assert(NPAD % B == 0, "NPAD must be a multiple of the pivot block");
    int pos = lane;
    R dg = R(1);  // the lane's U diagonal element once it has supplied a pivot
    bool ok = true;
    // blocks of B pivot columns; each block ends by rotating the row left by B, so the next
    // block's pivot columns sit in a[0..B-1].  All NPAD / B rotations are made, which brings
    // column j back to a[j] for the back substitution.  Up to NPAD = 40 the block loop is
    // unrolled, which turns the rotations into register renaming and the skips into constants;
    // larger rows keep it rolled so that the code stays within the instruction cache.
    constexpr int kBlkUnroll = NPAD <= 40 ? NPAD / B : 1;
#pragma unroll kBlkUnroll
    for (int blk = 0; blk < NPAD / B; ++blk) {
        if (B * blk < N) {
#pragma unroll
            for (int kk = 0; kk < B; ++kk) {
                const int k = B * blk + kk;
                if (k < N) {
                    const int w = pivot_lane<R>((R)fabs(a[kk]), pos >= k && lane < N, pos);
                    const int p = rdlane(pos, w);
                    pos = (lane == w) ? k : (pos == k ? p : pos);
                    const R piv = rdlane(a[kk], w);
                    ok = ok && piv != R(0);
                    const R yk = rdlane(bb, w);
                    dg = (lane == w) ? piv : dg;
                    const bool elim = pos > k;
                    const R l = elim ? a[kk] * rpiv_of(piv) : R(0);
                    bb = fma(-l, yk, bb);
                    // pivot row from the pivot lane's registers, eight columns at a time;
                    // register positions from NPAD - B blk on hold columns already eliminated
                    // (rotated in from the front) and are skipped eight at a time.  Rows that
                    // have supplied a pivot take l = 0 and stay as they are.
#pragma unroll
                    for (int j0 = kk + 1; j0 < NPAD; j0 += 8) {
                        if (j0 >= NPAD - B * blk) break;
                        R pr[8];
#pragma unroll
                        for (int j = j0; j < j0 + 8 && j < NPAD; ++j) pr[j - j0] = rdlane(a[j], w);
#pragma unroll
                        for (int j = j0; j < j0 + 8 && j < NPAD; ++j) a[j] = fma(-l, pr[j - j0], a[j]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        }
        R t[B];
#pragma unroll
        for (int j = 0; j < B; ++j) t[j] = a[j];
#pragma unroll
        for (int j = 0; j + B < NPAD; ++j) a[j] = a[j + B];
#pragma unroll
        for (int j = 0; j < B; ++j) a[NPAD - B + j] = t[j];
    }
    // back substitution, columns from the last: the lane holding U row k forms
    // x_k = y_k / u_kk, and every row above k removes u_ik x_k from its y_i
    const R rdg = R(1) / dg;
    R xl = R(0);
#pragma unroll
    for (int k = NPAD - 1; k >= 0; --k) {
        if (k < N) {
            const int o = __builtin_ctzll(__ballot(pos == k));
            const R xk = rdlane(bb, o) * rdlane(rdg, o);
            xl = (lane == k) ? xk : xl;
            if (pos < k) bb = fma(-a[k], xk, bb);
        }
    }
    x = xl;
    return ok;
}

// 16 x 16 x 4 FP64 matrix instruction: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator register r of lane l holds output column l % 16 and row 4 r + l / 16
template <typename R> struct Mfma;
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int lane) { return 4 * r + (lane >> 4); }
};

// 1/p from the hardware reciprocal refined by Newton steps (within an ulp for normal p)
__device__ __forceinline__ double recip(double p)
{
    double y = __builtin_amdgcn_rcp(p);
    y = fma(y, fma(-p, y, 1.0), y);
    return fma(y, fma(-p, y, 1.0), y);
}

// Gaussian elimination with partial pivoting on the augmented Newton matrix [A | b] in the
// wavefront's LDS: row i at M + i S (S odd), N rows, b in column N.  Right-looking, blocked by
// four columns, with LAPACK's order of row exchanges:
//   * panel: its four columns (and b when it lies in the panel) are held in registers, one row
//     per lane, for its four pivot steps; rows keep their lanes and carry their current
//     position.  Step k takes the largest |a_ik| over positions k..N-1 (ties to the lowest
//     position), exchanges positions k and p (right of the panel in LDS, by one column per
//     lane), forms the multipliers in column k and updates the panel's other columns with the
//     pivot row's entries broadcast by readlane; each row is then written back at its final
//     position;
//   * the pivot rows right of the panel, U12 = L11^-1 A12 (one column per lane);
//   * the rest, A22 -= L21 U12, on the matrix instructions in 16 x 16 tiles with k = 4.
// Columns left of the panel are not exchanged: b is eliminated with the matrix, so the
// multipliers stored there are not read again.  Back substitution from U and y (column N)
// follows.  Lane k returns x_k (lanes >= N: 0); false on an exactly zero pivot.
template <int NPAD, typename R>
__device__ __forceinline__ bool lu_solve_lds(R *M, int S, int N, int lane, R &x)
{
    typedef Mfma<R> MF;
    constexpr int TQ = (NPAD - 3 + 15) / 16;  // column tiles right of a panel (columns 4..N)
    bool ok = true;
    R rdiag = R(1);  // lane k: 1 / u_kk
    const int g = lane >> 4, c16 = lane & 15;
    const int lr = lane < N ? lane : N - 1;  // a lane's row for reads (lanes >= N read a real row)
    R *Mr = M + lr * S;
    for (int c0 = 0; c0 < N; c0 += 4) {
        // the panel's four columns (and b when it lies in the panel) in registers, one row per
        // lane; the pivot row's entries reach the other lanes by readlane
        R P[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) P[jj] = (c0 + jj <= N) ? Mr[c0 + jj] : R(0);
        // rows do not move between lanes during the panel: pos is a row's current position,
        // and the write-back below puts each row at its final one
        int pos = lane;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = c0 + kk;
            if (k >= N) break;
            const bool cand = pos >= k && lane < N;
            const R v = cand ? P[kk] : R(0);
            const int w = pivot_lane<R>((R)fabs(v), cand, pos);  // the lane holding the pivot row
            const int p = rdlane(pos, w);
            const R piv = rdlane(v, w);
            ok = ok && piv != R(0);
            if (p != k) {
                // right of the panel the rows at positions k and p are exchanged in LDS, one
                // column per lane (later exchanges of the panel keep LDS order)
                const int j = c0 + 4 + lane;
                if (j <= N) {
                    R *a = M + k * S + j, *b = M + p * S + j;
                    const R rk = *a, rpv = *b;
                    *a = rpv;
                    *b = rk;
                }
            }
            pos = (lane == w) ? k : (pos == k ? p : pos);
            const R rp = recip(piv);
            rdiag = (lane == k) ? rp : rdiag;
            const bool below = pos > k && lane < N;
            const R l = P[kk] * rp;
            P[kk] = below ? l : P[kk];
#pragma unroll
            for (int jj = kk + 1; jj < 4; ++jj) {
                if (c0 + jj > N) break;
                const R u = rdlane(P[jj], w);
                P[jj] = below ? fma(-l, u, P[jj]) : P[jj];
            }
        }
        if (lane < N) {
            R *Mp = M + pos * S;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
                if (c0 + jj <= N) Mp[c0 + jj] = P[jj];
        }
        wave_sync();
        const int t0 = c0 + 4;
        if (t0 > N) break;  // that panel held the last columns and b
        {   // U12: forward substitution with the panel's unit lower triangle, one column per lane
            const int j = t0 + lane;
            const bool col = j <= N;
            const int jj = col ? j : N;
            const R *Pr = M + c0 * S;
            R u0 = Pr[jj], u1 = Pr[S + jj], u2 = Pr[2 * S + jj], u3 = Pr[3 * S + jj];
            const R l10 = Pr[S + c0], l20 = Pr[2 * S + c0], l21 = Pr[2 * S + c0 + 1];
            const R l30 = Pr[3 * S + c0], l31 = Pr[3 * S + c0 + 1], l32 = Pr[3 * S + c0 + 2];
            u1 = fma(-l10, u0, u1);
            u2 = fma(-l21, u1, fma(-l20, u0, u2));
            u3 = fma(-l32, u2, fma(-l31, u1, fma(-l30, u0, u3)));
            if (col) {
                R *Q = M + c0 * S + j;
                Q[S] = u1;
                Q[2 * S] = u2;
                Q[3 * S] = u3;
            }
            wave_sync();
        }
        // trailing rows t0..N-1, columns t0..N: C -= L21 U12, one 16 x 16 tile per instruction
        for (int r0 = t0; r0 < N; r0 += 16) {
            const int ra = r0 + c16;
            const R a0 = M[(ra < N ? ra : N - 1) * S + c0 + g];
            const R av = ra < N ? -a0 : R(0);
            int crow[4];
            bool rin[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + MF::row(r, lane);
                rin[r] = row < N;
                crow[r] = (rin[r] ? row : N - 1) * S;
            }
            // the row of tiles: all operand and accumulator loads first, then the instructions,
            // then the stores
            typename MF::v4 acc[TQ];
            R bv[TQ];
#pragma unroll
            for (int tq = 0; tq < TQ; ++tq) {
                const int qb = t0 + 16 * tq + c16;
                if (t0 + 16 * tq > N) break;
                const int qc = qb <= N ? qb : N;
                const R b0 = M[(c0 + g) * S + qc];
                bv[tq] = qb <= N ? b0 : R(0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[tq][r] = M[crow[r] + qc];
            }
#pragma unroll
            for (int tq = 0; tq < TQ; ++tq) {
                if (t0 + 16 * tq > N) break;
                acc[tq] = MF::op(av, bv[tq], acc[tq]);
            }
#pragma unroll
            for (int tq = 0; tq < TQ; ++tq) {
                const int qb = t0 + 16 * tq + c16;
                if (t0 + 16 * tq > N) break;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (rin[r] && qb <= N) M[crow[r] + qb] = acc[tq][r];
            }
        }
        wave_sync();
    }
    // back substitution: x_k = y_k / u_kk, then every row above k removes u_ik x_k from y_i
    R y = lane < N ? Mr[N] : R(0);
    R xl = R(0);
    for (int k = N - 1; k >= 0; --k) {
        const R uik = Mr[k];
        const R xk = rdlane(y * rdiag, k);  // lane k's y is final here
        xl = (lane == k) ? xk : xl;
        y = (lane < k) ? fma(-uik, xk, y) : y;
    }
    x = xl;
    return ok;
}

struct StepCtl {
    double rtol, atol_Y, atol_T, y_neg;
    int k_max;
    bool point_implicit;   // accept the first (linearised) update as it is
    double diverge_ratio;  // > 0: fail an attempt whose update norm grows by more than this
};

// One backward-Euler sub-step of size h.  xs (lane i: x_i) is updated on success.
template <int NPAD, bool F32, bool PK>
__device__ __forceinline__ bool substep(const WaveTables &t, const Lds &L, int lane, double rho, double e0,
                                        double &xs, double h, const StepCtl &c, int &iters, double Ms,
                                        double invMs)
{
    const int ns = t.ns, N = ns + 1, JS = j_stride(NPAD);
    double xk = xs;
    double r_prev = -1.0;  // weighted norm of the previous update
    for (int k = 0; k < c.k_max; ++k) {
        ++iters;
        eval<NPAD, PK>(t, L, lane, rho, xk, Ms, invMs);
        bool ok;
        double d;
        if constexpr (F32) {
            // the Newton matrix row I - hJ, formed in place (columns N.. stay zero), then loaded,
            // scaled by its largest magnitude and rounded to FP32 for the register elimination
            double bi = 0.0;
            double arow[NPAD];
            bool bad = false;
            if (lane < N) {
                bi = -((xk - xs) - h * L.W[lane]);
                bad = !__builtin_isfinite(bi);
                double *Jr = L.J + (size_t)lane * JS;
#pragma unroll 4
                for (int j = 0; j < N; ++j) {
                    const double v = (j == lane ? 1.0 : 0.0) - h * Jr[j];
                    Jr[j] = v;
                    bad = bad || !__builtin_isfinite(v);
                }
#pragma unroll
                for (int j = 0; j < NPAD; ++j) arow[j] = j < N ? Jr[j] : 0.0;
            } else {
#pragma unroll
                for (int j = 0; j < NPAD; ++j) arow[j] = 0.0;
            }
            if (__any(bad)) return false;
            wave_sync();  // J and f are read before the next evaluation clears them
            float af[NPAD];
            double m = 0.0;
#pragma unroll
            for (int j = 0; j < NPAD; ++j) m = fmax(m, fabs(arow[j]));
            const double sc = (lane < N) ? 1.0 / m : 0.0;
#pragma unroll
            for (int j = 0; j < NPAD; ++j) af[j] = (float)(arow[j] * sc);
            float xf;
            ok = lu_solve<NPAD, float>(af, (float)(bi * sc), N, lane, xf);
            d = (double)xf;
        } else {
            // the augmented Newton matrix [I - hJ | b] in place of J, one row per lane
            bool bad = false;
            if (lane < N) {
                const double bi = -((xk - xs) - h * L.W[lane]);
                bad = !__builtin_isfinite(bi);
                double *Jr = L.J + (size_t)lane * JS;
#pragma unroll 4
                for (int j = 0; j < N; ++j) {
                    const double v = (j == lane ? 1.0 : 0.0) - h * Jr[j];
                    Jr[j] = v;
                    bad = bad || !__builtin_isfinite(v);
                }
                Jr[N] = bi;
            }
            if (__any(bad)) return false;
            wave_sync();
            ok = lu_solve_lds<NPAD, double>(L.J, JS, N, lane, d);
        }
        if (!ok) return false;
        wave_sync();
        xk += d;
        const double atol = (lane < ns) ? c.atol_Y : c.atol_T;
        if (__any(lane < N && !__builtin_isfinite(xk))) return false;
        const double T = rdlane(xk, ns);
        if (T < kTmin || T > kTmax) return false;
        const bool conv = c.point_implicit || __all(lane >= N || fabs(d) <= atol + c.rtol * fabs(xk));
        if (!conv && c.diverge_ratio > 0.0) {  // Newton diverging: abandon the attempt
            const double r = wave_max(lane < N ? fabs(d) / (atol + c.rtol * fabs(xk)) : 0.0);
            if (r_prev >= 0.0 && r > c.diverge_ratio * r_prev) return false;
            r_prev = r;
        }
        if (conv) {
            if (!c.point_implicit && __any(lane < ns && xk < -c.y_neg)) return false;
            double Tn;
            if (!invert_T(t, lane, (lane < ns) ? xk : 0.0, e0, T, Tn)) return false;
            xs = (lane == ns) ? Tn : xk;
            return true;
        }
    }
    return false;
}

template <int NPAD, bool F32, bool PK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) wave_kernel(WaveTables t, AdvanceArgs a, int wpb)
{
    extern __shared__ double smem[];
    const int lane = threadIdx.x & (kW - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);
    const int ns = t.ns, N = ns + 1;
    const Lds L = lds_map<PK>(smem + (size_t)wid * lds_doubles(N, t.ntb, NPAD), N, NPAD);
    const StepCtl c{a.rtol, a.atol_Y, a.atol_T, a.y_neg, a.k_max, a.point_implicit != 0, a.diverge_ratio};
    const double Ms = lane < ns ? t.M[lane] : 1.0;
    const double invMs = 1.0 / Ms;
    // one cell per wavefront; the hardware dispatcher hands out blocks as earlier ones
    // retire, which balances cells that need very different numbers of Newton iterations
    const long long gcell = (long long)blockIdx.x * wpb + wid;
    if (gcell >= a.total) return;
    int j = 0;
    while (j + 1 < a.nspan && a.span[j + 1].start <= gcell) ++j;
    const long long pos = gcell - a.span[j].start;
    long long cell = pos;
    if (a.span[j].order) {
        const long long c = a.span[j].order[pos];
        if ((unsigned long long)c < (unsigned long long)a.span[j].n) cell = c;
    }
    const double dt = a.span[j].dt;
    const Arena ar = arena_at(a.span[j].base, a.span[j].n, ns);
    const long long ld = a.span[j].n;
    const double rho = ar.rho[cell];
    const double e0 = ar.e0[cell];
    double xs = 0.0;
    if (lane < ns) xs = ar.Y[(size_t)lane * ld + cell];
    else if (lane == ns) xs = ar.T[cell];
    const double T0 = rdlane(xs, ns);
    const bool bad_in = __any(lane < N && !__builtin_isfinite(xs)) || !__builtin_isfinite(rho) ||
                        !(rho > 0.0) || !__builtin_isfinite(e0) || !__builtin_isfinite(dt) ||
                        !(dt >= 0.0) || T0 < kTmin || T0 > kTmax;
    // dyadic sub-stepping in ticks of dt 2^-Lc (see the lane layout for the rule)
    const bool adapt = a.L_forced < 0;
    const int Lc = adapt ? a.L_max : a.L_forced;
    const unsigned long long end = 1ull << Lc;
    unsigned long long tt = bad_in ? end : 0ull;
    int l = adapt ? 0 : a.L_forced;
    int iters = 0, level = bad_in ? 0 : l, st = bad_in ? 3 : 0;
    bool failed = false;
    unsigned long long hsh = 0xcbf29ce484222325ull;  // FNV-1a of the sub-step attempts
    ScheduleTrace tr;
    tr.start(a.trace, a.trace_words, a.span[j].start + cell);
    while (tt < end) {
        if (iters >= a.max_iters) { st = 2; break; }
        const double h = ldexp(dt, -l);
        const bool ok = substep<NPAD, F32, PK>(t, L, lane, rho, e0, xs, h, c, iters, Ms, invMs);
        hsh = (hsh ^ (unsigned long long)(2 * l + (ok ? 1 : 0))) * 0x100000001b3ull;
        tr.add(ok, lane);
        if (ok) {
            tt += 1ull << (Lc - l);
            if (adapt && l > 0 && (tt & ((1ull << (Lc - l + 1)) - 1ull)) == 0ull) --l;
        } else {
            if (!adapt) { st = 2; break; }
            failed = true;
            ++l;
            if (l > level) level = l;
            if (l > a.L_max) { level = a.L_max; st = 2; break; }
        }
    }
    if (st == 0 && failed) st = 1;
    if (st < 2) {
        if (lane < ns) ar.Y[(size_t)lane * ld + cell] = xs;
        else if (lane == ns) ar.T[cell] = xs;
    }
    if (lane == 0) {
        ar.status[cell] = st;
        ar.level[cell] = level;
        ar.iters[cell] = iters;
        ar.sched[cell] = hsh;
    }
    tr.finish(lane);
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void energy_kernel(WaveTables t, long long n, long long ld, const double *T,
                              const double *Y, double *e0)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double Ti = T[i];
    double e = 0.0;
    for (int s = 0; s < t.ns; ++s) {
        const Thermo th = thermo(t, s, Ti, 1.0 / Ti, 0.0);
        e = fma(Y[(size_t)s * ld + i], 8.31446261815324e3 / t.M[s] * Ti * (th.h - 1.0), e);
    }
    e0[i] = e;
}

// ---- conserved-variable adapter (one thread per cell) -----------------------------------------
__device__ __forceinline__ void cell_energy(const WaveTables &t, long long ld, long long i, const double *Y,
                                            double T, double &e, double &cv)
{
    e = 0.0;
    cv = 0.0;
    const double iT = 1.0 / T;
    for (int s = 0; s < t.ns; ++s) {
        const Thermo th = thermo(t, s, T, iT, 0.0);
        const double rm = 8.31446261815324e3 / t.M[s];
        const double y = Y[(size_t)s * ld + i];
        e = fma(y, rm * T * (th.h - 1.0), e);
        cv = fma(y, rm * (th.cp - 1.0), cv);
    }
}

// In: Y holds rho_s, e0 holds E_sens and T the starting temperature.  Out: rho, Y, e0 and T of
// the cell (T = NaN when e(Y, T) = e0 has no root in range).
__global__ void conserved_in_kernel(WaveTables t, long long n, long long ld, double *rho, double *T,
                                    double *Y, double *e0, int have_guess)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = 0.0;
    for (int s = 0; s < t.ns; ++s) r += Y[(size_t)s * ld + i];
    const double ir = 1.0 / r;
    double ef = 0.0;
    for (int s = 0; s < t.ns; ++s) {
        const double y = Y[(size_t)s * ld + i] * ir;
        Y[(size_t)s * ld + i] = y;
        ef = fma(y, t.ef[s], ef);
    }
    const double e_t = e0[i] * ir + ef;
    rho[i] = r;
    e0[i] = e_t;
    // Newton on e(Y, T) = e0 from the start value, then bisection on [kTmin, kTmax]
    double Tk = have_guess ? T[i] : 1500.0;
    if (!(Tk >= kTmin && Tk <= kTmax)) Tk = 1500.0;
    double Tout = __builtin_nan("");
    bool done = false;
    if (t.ns < 32) {
        // Within one NASA-7 range per species, e(Y, T) and c_v are polynomials in T with the
        // mass-weighted coefficients B_k = sum_s Y_s R_s a_sk: e = B_5 + T (B_0 + ... + T B_4 / 5)
        // - rR T and c_v = B_0 + T (B_1 + ... + T B_4) - rR.  The B_k are summed again only when
        // T crosses a species' switch temperature (a bit per species, set below it).
        double B[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, rR = 0.0;
        for (int s = 0; s < t.ns; ++s) rR = fma(Y[(size_t)s * ld + i], 8.31446261815324e3 / uniform_table(t.M)[s], rR);
        unsigned used = ~0u;  // no valid choice yet (fewer than 32 species)
        for (int it = 0; it < 20 && !done; ++it) {
            unsigned lo = 0;
            for (int s = 0; s < t.ns; ++s) lo |= (Tk < uniform_table(t.Tmid)[s] ? 1u : 0u) << s;
            if (lo != used) {
                used = lo;
#pragma unroll
                for (int k = 0; k < 6; ++k) B[k] = 0.0;
                for (int s = 0; s < t.ns; ++s) {
                    const auto *a = uniform_table(t.nasa) + 14 * s;
                    const bool l = (lo >> s) & 1u;
                    const double w = Y[(size_t)s * ld + i] * (8.31446261815324e3 / uniform_table(t.M)[s]);
#pragma unroll
                    for (int k = 0; k < 6; ++k) B[k] = fma(w, l ? a[k] : a[7 + k], B[k]);
                }
            }
            const double C = fma(Tk, fma(Tk, fma(Tk, fma(Tk, B[4], B[3]), B[2]), B[1]), B[0]);
            const double H = fma(Tk, fma(Tk, fma(Tk, fma(Tk, fma(Tk, B[4] * 0.2, B[3] * 0.25), B[2] * (1.0 / 3.0)),
                                                  B[1] * 0.5), B[0]), B[5]);
            const double e = H - rR * Tk, cv = C - rR;
            if (!(cv > 0.0)) break;
            const double dT = (e - e_t) / cv;
            Tk -= dT;
            if (!__builtin_isfinite(Tk) || Tk < kTmin || Tk > kTmax) break;
            if (fabs(dT) <= 1e-13 * Tk) { Tout = Tk; done = true; }
        }
    } else {
        for (int it = 0; it < 20 && !done; ++it) {
            double e, cv;
            cell_energy(t, ld, i, Y, Tk, e, cv);
            if (!(cv > 0.0)) break;
            const double dT = (e - e_t) / cv;
            Tk -= dT;
            if (!__builtin_isfinite(Tk) || Tk < kTmin || Tk > kTmax) break;
            if (fabs(dT) <= 1e-13 * Tk) { Tout = Tk; done = true; }
        }
    }
    if (!done) {
        double lo = kTmin, hi = kTmax, e, cv;
        cell_energy(t, ld, i, Y, lo, e, cv);
        const double flo = e - e_t;
        cell_energy(t, ld, i, Y, hi, e, cv);
        const double fhi = e - e_t;
        if (flo <= 0.0 && fhi >= 0.0) {
            for (int it = 0; it < 200 && hi - lo > 1e-13 * lo; ++it) {
                const double mid = 0.5 * (lo + hi);
                cell_energy(t, ld, i, Y, mid, e, cv);
                if (e - e_t > 0.0) hi = mid; else lo = mid;
            }
            Tout = 0.5 * (lo + hi);
        }
    }
    T[i] = Tout;
}

__global__ void conserved_out_kernel(WaveTables t, long long n, long long ld, const double *rho,
                                     const double *Y, const double *e0, double *rho_s, double *E_sens)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double r = rho[i];
    double ef = 0.0;
    for (int s = 0; s < t.ns; ++s) {
        const double y = Y[(size_t)s * ld + i];
        rho_s[(size_t)s * n + i] = r * y;
        ef = fma(y, t.ef[s], ef);
    }
    E_sens[i] = r * (e0[i] - ef);
}

template <int NPAD, bool F32>
hipError_t launch_t(const WaveTables &t, const AdvanceArgs &a, int wpb, int grid, hipStream_t s)
{
    const int N = t.ns + 1;
    const size_t lds = sizeof(double) * lds_doubles(N, t.ntb, NPAD) * wpb;
    if (lds > 65536) return hipErrorInvalidConfiguration;
    if (packed_vectors(N, NPAD))
        hipLaunchKernelGGL((wave_kernel<NPAD, F32, true>), dim3(grid), dim3(kW * wpb), lds, s, t, a, wpb);
    else
        hipLaunchKernelGGL((wave_kernel<NPAD, F32, false>), dim3(grid), dim3(kW * wpb), lds, s, t, a, wpb);
    return hipGetLastError();
}

}  // namespace

int wave_npad(int n)
{
    const int sizes[] = {16, 24, 32, 40, 48, 64};
    for (int p : sizes) if (n <= p) return p;
    return -1;
}

size_t wave_lds_bytes(const WaveTables &t, bool)
{
    const int N = t.ns + 1, p = wave_npad(N);
    return p < 0 ? 0 : sizeof(double) * lds_doubles(N, t.ntb, p);
}

hipError_t launch_wave(const WaveTables &t, const AdvanceArgs &a, bool f32, int wpb, int grid,
                       hipStream_t s)
{
    const int N = t.ns + 1;
#define KIN_CASE(P)                                                                   \
    case P:                                                                           \
        return f32 ? launch_t<P, true>(t, a, wpb, grid, s) : launch_t<P, false>(t, a, wpb, grid, s);
    switch (wave_npad(N)) {
        KIN_CASE(16)
        KIN_CASE(24)
        KIN_CASE(32)
        KIN_CASE(40)
        KIN_CASE(48)
        KIN_CASE(64)
    default:
        return hipErrorInvalidValue;
    }
#undef KIN_CASE
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_energy(const WaveTables &t, long long n, long long ld, const double *T,
                         const double *Y, double *e0, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    hipLaunchKernelGGL(energy_kernel, dim3((unsigned)grid), dim3(block), 0, s, t, n, ld, T, Y, e0);
    return hipGetLastError();
}

hipError_t launch_conserved_in(const WaveTables &t, long long n, long long ld, double *rho, double *T,
                               double *Y, double *e0, bool have_guess, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    hipLaunchKernelGGL(conserved_in_kernel, dim3((unsigned)grid), dim3(block), 0, s, t, n, ld, rho, T, Y,
                       e0, have_guess ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_conserved_out(const WaveTables &t, long long n, long long ld, const double *rho,
                                const double *Y, const double *e0, double *rho_s, double *E_sens,
                                hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    hipLaunchKernelGGL(conserved_out_kernel, dim3((unsigned)grid), dim3(block), 0, s, t, n, ld, rho, Y,
                       e0, rho_s, E_sens);
    return hipGetLastError();
}

}  // namespace kin
