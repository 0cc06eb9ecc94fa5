// kin_wave.hip -- table-driven kernels: the wave layout (one cell per 64-wide wavefront, one
// row of the Newton matrix per lane) and the initial-energy kernel.
//
// Method (Le & Cambier, arXiv:1110.4903): rates from the Arrhenius law, reverse rates from
// the equilibrium constant and third-body sums (Sec. 3.2); the point-implicit system
// (I - h dOmega/dQ) dQ = -G (Sec. 3.2, Eq. "kinetics") iterated as Newton's method on
// backward Euler; Gaussian elimination with partial pivoting per cell (Sec. 4.2).  The paper
// stored a cell's Jacobian either in global memory or in one thread block's shared memory;
// here a cell owns one wavefront: lanes evaluate reactions 64 at a time, species rows are
// accumulated in LDS, and each lane then holds one matrix row in registers for the
// elimination, with the pivot row broadcast through LDS and the pivot search done by a
// butterfly of cross-lane shuffles.  Wavefronts of a block never synchronise with each
// other, so cells with different iteration counts do not wait for one another.
#include <hip/hip_runtime.h>

#include "kin_internal.h"

namespace kin {

namespace {

constexpr double kTmin = 200.0, kTmax = 6000.0;
constexpr int kW = 64;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kW);
    return v;
}

__device__ __forceinline__ double bcast(double v, int lane)
{
    return __shfl(v, lane, kW);
}

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

// Per-wave LDS layout (in doubles).  JS = NPAD + 1 (row stride of the Jacobian).
struct Lds {
    double *J;     // [N][JS]
    double *c;     // [NPAD] concentrations
    double *g;     // [NPAD] g/RT
    double *h;     // [NPAD] h/RT
    double *ek;    // [NPAD] e_s (J/kg)
    double *cvk;   // [NPAD] cv_s (J/kg/K)
    double *f;     // [NPAD] right-hand side
    double *sol;   // [NPAD] solution exchange
    double *invM;  // [NPAD]
    double *cq;    // [9][kChunk] chunk buffer: q, dqT, D, dq[6]
    double *Mc;    // [ntb] third-body concentrations
    double *prow;  // [NPAD + 2] pivot row (FP64 or FP32 view)
};

template <int NPAD>
__host__ __device__ __forceinline__ size_t lds_doubles(int N, int ntb)
{
    return (size_t)N * (NPAD + 1) + 8 * NPAD + 9 * kChunk + (size_t)((ntb + 1) & ~1) + NPAD + 2;
}

template <int NPAD>
__device__ __forceinline__ Lds lds_map(double *base, int N, int ntb)
{
    Lds L;
    double *p = base;
    L.J = p; p += (size_t)N * (NPAD + 1);
    L.c = p; p += NPAD;
    L.g = p; p += NPAD;
    L.h = p; p += NPAD;
    L.ek = p; p += NPAD;
    L.cvk = p; p += NPAD;
    L.f = p; p += NPAD;
    L.sol = p; p += NPAD;
    L.invM = p; p += NPAD;
    L.cq = p; p += 9 * kChunk;
    L.Mc = p; p += (ntb + 1) & ~1;
    L.prow = p;
    return L;
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

__device__ __forceinline__ double cpow_nu(double c, int nu)
{
    return (nu == 1) ? c : (nu == 2 ? c * c : c * c * c);
}

// f = dx/dt and J = df/dx of the cell at x (lane i holds x_i).  Leaves J in L.J (rows
// 0..N-1) and f in L.f.
//
// Per pass of 64 reactions (one per lane) the rates, net progress, its T-derivative and its
// derivatives with respect to the participating concentrations go to the chunk buffer; then
// lane s, owner of Jacobian row s, gathers the chunk's contributions to its row from a
// precomputed list of (reaction, participant, column, coefficient) entries, and lane k adds
// column k of the dense third-body terms nu_rs (M_s / M_k) eff_rk (q_f - q_b).
template <int NPAD>
__device__ __forceinline__ void eval(const WaveTables &t, const Lds &L, int lane, double rho, double xs)
{
    const int ns = t.ns, N = ns + 1, JS = NPAD + 1;
    const double T = bcast(xs, ns);
    const double iT = 1.0 / T, lT = log(T);
    const double rc = 1e-3 * rho, irc = 1.0 / rc;
    const double lPaRT = t.lnPaR - lT;  // ln(P_atm / (R T)), CGS
    for (int k = lane; k < N * JS; k += kW) L.J[k] = 0.0;
    double cvk = 0.0, dcvk = 0.0, ek = 0.0;
    if (lane < ns) {
        const Thermo th = thermo(t, lane, T, iT, lT);
        const double invM = 1.0 / t.M[lane];
        const double rm = 8.31446261815324e3 * invM;
        L.c[lane] = xs * (rc * invM);
        L.g[lane] = th.h - th.s;
        L.h[lane] = th.h;
        ek = rm * T * (th.h - 1.0);
        cvk = rm * (th.cp - 1.0);
        dcvk = rm * th.dcp;
        L.ek[lane] = ek;
        L.cvk[lane] = cvk;
        L.invM[lane] = invM;
    }
    wave_sync();
    // third-body concentrations [M]_r = sum_s eff_rs c_s, one reaction per lane
    for (int r = lane; r < t.ntb; r += kW) {
        double acc = 0.0;
        for (int s = 0; s < ns; ++s) acc = fma(t.effT[(size_t)s * t.ntb + r], L.c[s], acc);
        L.Mc[r] = acc;
    }
    wave_sync();
    double w = 0.0, jt = 0.0;
    double *const Q = L.cq, *const QT = L.cq + kChunk, *const DD = L.cq + 2 * kChunk;
    double *const DQ = L.cq + 3 * kChunk;
    const double Ms = (lane < ns) ? t.M[lane] : 0.0;
    for (int cb = 0; cb < t.nchunk; ++cb) {
        const int r = cb * kChunk + lane;
        if (r < t.nr) {
            const RxnRec x = t.rxc[r];
            const double *rd = t.rxd + (size_t)r * 4;
            const double b = rd[1], Ta = rd[2], dnu = rd[3];
            const double lkf = fma(-Ta, iT, fma(b, lT, rd[0]));
            const double kf = exp(lkf);
            const double dlkf = fma(Ta, iT, b) * iT;
            double cr[3], cpd[3];
            double pf = kf;
            for (int j = 0; j < x.nreac; ++j) {
                cr[j] = L.c[x.reac_sp[j]];
                pf *= cpow_nu(cr[j], x.reac_nu[j]);
            }
            double kb = 0.0, pb = 0.0, dlKc = 0.0;
            if (x.rev) {
                double sg = 0.0, sh = 0.0;
                for (int j = 0; j < x.npart; ++j) {
                    const double nu = (double)x.part_nu[j];
                    sg = fma(nu, L.g[x.part_sp[j]], sg);
                    sh = fma(nu, L.h[x.part_sp[j]], sh);
                }
                const double lKc = dnu * lPaRT - sg;
                kb = exp(lkf - lKc);
                dlKc = (sh - dnu) * iT;
                pb = kb;
                for (int j = 0; j < x.nprod; ++j) {
                    cpd[j] = L.c[x.prod_sp[j]];
                    pb *= cpow_nu(cpd[j], x.prod_nu[j]);
                }
            }
            const double Mc = (x.tb >= 0) ? L.Mc[x.tb] : 1.0;
            const double D = pf - pb;
            Q[lane] = Mc * D;
            QT[lane] = Mc * (pf * dlkf - pb * (dlkf - dlKc));
            DD[lane] = D;
            for (int j = 0; j < x.npart; ++j) {
                const int sp = x.part_sp[j];
                // d/dc_sp of kf prod c^nu' minus d/dc_sp of kb prod c^nu''
                double gf = 0.0, gb = 0.0;
                for (int m = 0; m < x.nreac; ++m) {
                    if (x.reac_sp[m] != sp) continue;
                    const int nu = x.reac_nu[m];
                    double d = kf * (double)nu * (nu == 1 ? 1.0 : (nu == 2 ? cr[m] : cr[m] * cr[m]));
                    for (int o = 0; o < x.nreac; ++o)
                        if (o != m) d *= cpow_nu(cr[o], x.reac_nu[o]);
                    gf = d;
                }
                if (x.rev) {
                    for (int m = 0; m < x.nprod; ++m) {
                        if (x.prod_sp[m] != sp) continue;
                        const int nu = x.prod_nu[m];
                        double d = kb * (double)nu * (nu == 1 ? 1.0 : (nu == 2 ? cpd[m] : cpd[m] * cpd[m]));
                        for (int o = 0; o < x.nprod; ++o)
                            if (o != m) d *= cpow_nu(cpd[o], x.prod_nu[o]);
                        gb = d;
                    }
                }
                DQ[j * kChunk + lane] = Mc * (gf - gb);
            }
        }
        wave_sync();
        if (lane < ns) {
            const int *sp = t.sp_ptr + (size_t)lane * (t.nchunk + 1);
            for (int e = sp[cb]; e < sp[cb + 1]; ++e) {
                const int ent = t.sp_list[e];
                const int rl = ent >> 4;
                const double nu = (double)((ent & 15) - 8);
                w = fma(nu, Q[rl], w);
                jt = fma(nu, QT[rl], jt);
            }
            const int *ep = t.ent_ptr + (size_t)lane * (t.nchunk + 1);
            double *Jrow = L.J + (size_t)lane * JS;
            for (int e = ep[cb]; e < ep[cb + 1]; ++e) {
                const int ent = t.ent_list[e];
                const int rl = ent & 63, slot = (ent >> 6) & 7, k = (ent >> 9) & 63;
                const double nu = (double)(((ent >> 15) & 15) - 8);
                Jrow[k] = fma(nu * Ms * L.invM[k], DQ[slot * kChunk + rl], Jrow[k]);
            }
        }
        wave_sync();
        // dense third-body part, one Jacobian column per lane
        if (lane < ns) {
            for (int e = t.tb_ptr[cb]; e < t.tb_ptr[cb + 1]; ++e) {
                const int r2 = t.tb_list[e];
                const RxnRec x = t.rxc[r2];
                const double tk = DD[r2 - cb * kChunk] * t.effM[(size_t)x.tb * ns + lane];
                for (int j = 0; j < x.npart; ++j) {
                    if (!x.part_nu[j]) continue;
                    const int s2 = x.part_sp[j];
                    double *Jp = L.J + (size_t)s2 * JS + lane;
                    *Jp = fma((double)x.part_nu[j] * t.M[s2], tk, *Jp);
                }
            }
        }
        wave_sync();
    }
    // species rows of f and the temperature column
    double fs = 0.0;
    if (lane < ns) {
        const double ms = Ms * irc;
        fs = w * ms;
        L.J[(size_t)lane * JS + ns] = jt * ms;
        L.f[lane] = fs;
    }
    const double cv = wave_sum(lane < ns ? xs * cvk : 0.0);
    const double dcv = wave_sum(lane < ns ? xs * dcvk : 0.0);
    const double de = wave_sum(ek * fs);
    const double fT = -de / cv;
    const double icv = 1.0 / cv;
    wave_sync();
    // energy row: lane k < ns forms J[ns][k]; lane ns forms J[ns][ns]
    if (lane <= ns) {
        double acc = 0.0;
        if (lane < ns) {
            for (int s = 0; s < ns; ++s) acc = fma(L.ek[s], L.J[(size_t)s * JS + lane], acc);
            L.J[(size_t)ns * JS + lane] = -fma(fT, L.cvk[lane], acc) * icv;
        } else {
            for (int s = 0; s < ns; ++s)
                acc = fma(L.cvk[s], L.f[s], fma(L.ek[s], L.J[(size_t)s * JS + ns], acc));
            L.J[(size_t)ns * JS + ns] = -fma(fT, dcv, acc) * icv;
            L.f[ns] = fT;
        }
    }
    wave_sync();
}

// Gaussian elimination with partial pivoting, one row per lane.  Lane i < N enters with row i
// of A in a[] and b_i in bb; on return sol[0..N) in LDS holds the solution.  Pivot rule: the
// first (lowest current position) row of largest |a_ik| among rows not yet used.  Returns
// false on an exactly zero pivot.
template <int NPAD, typename R>
__device__ __forceinline__ bool lu_solve(R (&a)[NPAD], R bb, int N, int lane, const Lds &L)
{
    R *prow = reinterpret_cast<R *>(L.prow);
    int pos = lane;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NPAD; ++k) {
        if (k < N) {
            R v = (pos >= k) ? (R)fabs(a[k]) : R(-1);
            int p = pos;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const R ov = __shfl_xor(v, off, kW);
                const int op = __shfl_xor(p, off, kW);
                const bool take = (ov > v) || (ov == v && op < p);
                v = take ? ov : v;
                p = take ? op : p;
            }
            ok = ok && (v > R(0));
            const bool is_piv = (pos == p);
            pos = is_piv ? k : (pos == k ? p : pos);
            if (is_piv) {
#pragma unroll
                for (int j = k; j < NPAD; ++j) prow[j] = a[j];
                prow[NPAD] = bb;
            }
            wave_sync();
            if (pos > k) {
                const R l = a[k] / prow[k];
#pragma unroll
                for (int j = k + 1; j < NPAD; ++j) a[j] = fma(-l, prow[j], a[j]);
                bb = fma(-l, prow[NPAD], bb);
            }
            wave_sync();
        }
    }
    // back substitution, one unknown per step
#pragma unroll
    for (int k = NPAD - 1; k >= 0; --k) {
        if (k < N) {
            if (pos == k) L.sol[k] = (double)(bb / a[k]);
            wave_sync();
            const R xk = (R)L.sol[k];
            if (pos < k) bb = fma(-a[k], xk, bb);
            wave_sync();
        }
    }
    return ok;
}

struct StepCtl {
    double rtol, atol_Y, atol_T, y_neg;
    int k_max;
};

// One backward-Euler sub-step of size h.  xs (lane i: x_i) is updated on success.
template <int NPAD, bool F32>
__device__ __forceinline__ bool substep(const WaveTables &t, const Lds &L, int lane, double rho, double e0,
                        double &xs, double h, const StepCtl &c, int &iters)
{
    const int ns = t.ns, N = ns + 1, JS = NPAD + 1;
    double xk = xs;
    for (int k = 0; k < c.k_max; ++k) {
        ++iters;
        eval<NPAD>(t, L, lane, rho, xk);
        double bi = 0.0;
        double arow[NPAD];
        bool bad = false;
        if (lane < N) {
            bi = -((xk - xs) - h * L.f[lane]);
            bad = !__builtin_isfinite(bi);
            const double *Jr = L.J + (size_t)lane * JS;
#pragma unroll
            for (int j = 0; j < NPAD; ++j) {
                const double v = (j < N) ? ((j == lane ? 1.0 : 0.0) - h * Jr[j]) : 0.0;
                arow[j] = v;
                bad = bad || !__builtin_isfinite(v);
            }
        } else {
#pragma unroll
            for (int j = 0; j < NPAD; ++j) arow[j] = 0.0;
        }
        if (__any(bad)) return false;
        bool ok;
        if (F32) {
            float af[NPAD];
            double m = 0.0;
#pragma unroll
            for (int j = 0; j < NPAD; ++j) m = fmax(m, fabs(arow[j]));
            const double s = (lane < N) ? 1.0 / m : 0.0;
#pragma unroll
            for (int j = 0; j < NPAD; ++j) af[j] = (float)(arow[j] * s);
            ok = lu_solve<NPAD, float>(af, (float)(bi * s), N, lane, L);
        } else {
            ok = lu_solve<NPAD, double>(arow, bi, N, lane, L);
        }
        if (!ok) return false;
        const double d = (lane < N) ? L.sol[lane] : 0.0;
        wave_sync();
        xk += d;
        const double atol = (lane < ns) ? c.atol_Y : c.atol_T;
        if (__any(lane < N && !__builtin_isfinite(xk))) return false;
        const double T = bcast(xk, ns);
        if (T < kTmin || T > kTmax) return false;
        const bool conv = __all(lane >= N || fabs(d) <= atol + c.rtol * fabs(xk));
        if (conv) {
            if (__any(lane < ns && xk < -c.y_neg)) return false;
            double Tn;
            if (!invert_T(t, lane, (lane < ns) ? xk : 0.0, e0, T, Tn)) return false;
            xs = (lane == ns) ? Tn : xk;
            return true;
        }
    }
    return false;
}

template <int NPAD, bool F32>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) wave_kernel(WaveTables t, AdvanceArgs a, int wpb)
{
    extern __shared__ double smem[];
    const int lane = threadIdx.x & (kW - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);
    const int ns = t.ns, N = ns + 1;
    const Lds L = lds_map<NPAD>(smem + (size_t)wid * lds_doubles<NPAD>(N, t.ntb), N, t.ntb);
    const StepCtl c{a.rtol, a.atol_Y, a.atol_T, a.y_neg, a.k_max};
    // one cell per wavefront; the hardware dispatcher hands out blocks as earlier ones
    // retire, which balances cells that need very different numbers of Newton iterations
    {
        const long long gcell = (long long)blockIdx.x * wpb + wid;
        if (gcell >= a.total) return;
        int j = 0;
        while (j + 1 < a.nspan && a.span[j + 1].start <= gcell) ++j;
        const long long cell = gcell - a.span[j].start;
        const double dt = a.span[j].dt;
        const Arena ar = arena_at(a.span[j].base, a.span[j].n, ns);
        const long long ld = a.span[j].n;
        const double rho = ar.rho[cell];
        const double e0 = ar.e0[cell];
        double xs = 0.0;
        if (lane < ns) xs = ar.Y[(size_t)lane * ld + cell];
        else if (lane == ns) xs = ar.T[cell];
        const double T0 = bcast(xs, ns);
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
        while (tt < end) {
            if (iters >= a.max_iters) { st = 2; break; }
            const double h = ldexp(dt, -l);
            const bool ok = substep<NPAD, F32>(t, L, lane, rho, e0, xs, h, c, iters);
            hsh = (hsh ^ (unsigned long long)(2 * l + (ok ? 1 : 0))) * 0x100000001b3ull;
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
    }
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

template <int NPAD>
size_t lds_bytes_host(int N, int ntb)
{
    return sizeof(double) * lds_doubles<NPAD>(N, ntb);
}

template <int NPAD, bool F32>
hipError_t launch_t(const WaveTables &t, const AdvanceArgs &a, int wpb, int grid, hipStream_t s)
{
    const size_t lds = lds_bytes_host<NPAD>(t.ns + 1, t.ntb) * wpb;
    hipLaunchKernelGGL((wave_kernel<NPAD, F32>), dim3(grid), dim3(kW * wpb), lds, s, t, a, wpb);
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
    const int N = t.ns + 1;
    switch (wave_npad(N)) {
    case 16: return lds_bytes_host<16>(N, t.ntb);
    case 24: return lds_bytes_host<24>(N, t.ntb);
    case 32: return lds_bytes_host<32>(N, t.ntb);
    case 40: return lds_bytes_host<40>(N, t.ntb);
    case 48: return lds_bytes_host<48>(N, t.ntb);
    default: return lds_bytes_host<64>(N, t.ntb);
    }
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

}  // namespace kin
