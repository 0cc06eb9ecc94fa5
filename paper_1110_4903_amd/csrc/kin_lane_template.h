// kin_lane_template.h -- device code of the lane layout: one cell per lane, the (Ns+1)^2
// Newton matrix held in registers.  Compiled at mechanism upload (hipRTC, gfx950) after the
// generated mechanism code, which defines KIN_NS, KIN_N, KIN_BLOCK and
//   kin_eval(rho, x, f, J)        f = dx/dt and J = df/dx of the constant-(rho, e) cell
//   kin_energy_cv(Y, T, e, cv)    mixture internal energy (J/kg) and c_v (J/kg/K)
// Every array below is indexed only by compile-time constants after unrolling, so the
// compiler keeps it in VGPRs.  Partial pivoting is done with selects (v_cndmask), since a
// register file cannot be indexed by a per-lane pivot row.
//
// Method (Le & Cambier, arXiv:1110.4903, Sec. 3.2, Eq. "kinetics"): the point-implicit
// system (I - h J) dx = -G with G = x - x_prev - h f(x), iterated as Newton's method on
// backward Euler; the dense solve is Gaussian elimination with partial pivoting (Sec. 4.2).

// One instance's share of the launch: global cells [start, start + n) live in the arena at
// base (layout below), advanced by dt; order (when not null) maps a position of the span to
// the cell taken there (cells expected to need more iterations first).
struct KinSpan {
    long long start, n;
    double dt;
    char *base;
    const int *order;
};
#define KIN_MAX_SPANS 64

struct KinLaneArgs {
    KinSpan span[KIN_MAX_SPANS];
    int nspan, ns;
    long long total;      // cells over all spans
    double rtol, atol_Y, atol_T, y_neg;
    int k_max, L_max, L_forced, max_iters;
    int point_implicit;   // 1: accept the first (linearised) update as it is
    double diverge_ratio; // > 0: fail an attempt whose update norm grows by more than this
    const double *K;      // the mechanism's constant table (KIN_NCONST values)
    unsigned long long *counter;  // next unclaimed global cell; zero at launch
    // diagnostic sub-step schedules (recorded only by a module compiled with KIN_TRACE): cell
    // at launch position g has trace[g * trace_words ...]: the attempt count, then accept bits
    unsigned long long *trace;
    int trace_words;
};

// Arena of an instance of n cells: rho[n] e0[n] T[n] Y[ns][n] sched[n] as 8-byte arrays, then
// status[n] level[n] iters[n] as 4-byte arrays, each array starting on a 256-byte boundary.
__device__ __forceinline__ size_t kin_al(size_t x) { return (x + 255) & ~(size_t)255; }
__device__ __forceinline__ double *kin_rho(char *b, long long n) { return (double *)b; }
__device__ __forceinline__ double *kin_e0(char *b, long long n) { return (double *)(b + kin_al(8 * (size_t)n)); }
__device__ __forceinline__ double *kin_T(char *b, long long n) { return (double *)(b + 2 * kin_al(8 * (size_t)n)); }
__device__ __forceinline__ double *kin_Y(char *b, long long n) { return (double *)(b + 3 * kin_al(8 * (size_t)n)); }
__device__ __forceinline__ unsigned long long *kin_sched(char *b, long long n)
{
    return (unsigned long long *)(b + (3 + KIN_NS) * kin_al(8 * (size_t)n));
}
__device__ __forceinline__ int *kin_stat(char *b, long long n, int which)  // 0 status, 1 level, 2 iters
{
    return (int *)(b + (4 + KIN_NS) * kin_al(8 * (size_t)n) + which * kin_al(4 * (size_t)n));
}

#define KIN_SCHED_SEED 0xcbf29ce484222325ull
#define KIN_SCHED_PRIME 0x100000001b3ull

// The constant table is read through a pointer the compiler cannot see through, once per
// use site: the scalar loads of K[] then stay next to their uses instead of being hoisted
// out of the Newton loop, which would pin hundreds of constants in SGPRs.
__device__ __forceinline__ kin_cptr kin_launder(const double *p)
{
    asm volatile("" : "+s"(p));
    return (kin_cptr)p;
}

// Unknown held at position i of the solved system: T first, then the species.
#define KIN_VAR(i) ((i) == 0 ? KIN_NS : (i) - 1)

#define KIN_T_MIN 200.0
#define KIN_T_MAX 6000.0

// Solve e(Y, T) = e0 for T: Newton on c_v > 0 from T0, bisection on [200, 6000] K if
// Newton leaves the range or does not settle in 20 steps.
__device__ __forceinline__ bool kin_invert_T(const double *Kp, const double (&x)[KIN_N], double e0,
                                             double T0, double &T_out)
{
    double T = T0;
    for (int it = 0; it < 20; ++it) {
        double e, cv;
        kin_energy_cv(kin_launder(Kp), x, T, e, cv);
        if (!(cv > 0.0)) break;
        const double dT = (e - e0) / cv;
        T -= dT;
        if (!__builtin_isfinite(T) || T < KIN_T_MIN || T > KIN_T_MAX) break;
        if (fabs(dT) <= 1e-13 * T) { T_out = T; return true; }
    }
    double lo = KIN_T_MIN, hi = KIN_T_MAX, e, cv;
    kin_energy_cv(kin_launder(Kp), x, lo, e, cv);
    const double flo = e - e0;
    kin_energy_cv(kin_launder(Kp), x, hi, e, cv);
    const double fhi = e - e0;
    if (!(flo <= 0.0 && fhi >= 0.0)) return false;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * lo; ++it) {
        const double mid = 0.5 * (lo + hi);
        kin_energy_cv(kin_launder(Kp), x, mid, e, cv);
        if (e - e0 > 0.0) hi = mid; else lo = mid;
    }
    T_out = 0.5 * (lo + hi);
    return true;
}

// In-register LU with partial pivoting (first row of largest |a_ik|), applied to the
// right-hand side as it goes, then back substitution.  R is the factorisation type; in FP32
// the pivoting is by threshold (below).  Returns false on an exactly zero pivot, or in FP32
// a non-finite one.
//
// The row exchange is done with selects, since a register file cannot be indexed by a
// per-lane row.  It is done row by row, and only for the rows that are some lane's pivot row
// in this column (a wavefront-uniform test per row): each lane exchanges with exactly one row,
// so the result is that of the exchange, and a wavefront pays for the rows its lanes use
// rather than for every row below the diagonal.  The reciprocal of each pivot replaces the
// pivot in U, for the multipliers and the back substitution alike.
template <typename R>
__device__ __forceinline__ bool kin_lu_solve(R (&A)[KIN_N][KIN_N], R (&b)[KIN_N])
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < KIN_N; ++k) {
        R amax = fabs(A[k][k]);
        int p = k;
#pragma unroll
        for (int i = k + 1; i < KIN_N; ++i) {
            const R v = fabs(A[i][k]);
            const bool gt = v > amax;
            amax = gt ? v : amax;
            p = gt ? i : p;
        }
        ok = ok && (amax != R(0)) && (sizeof(R) == 8 || __builtin_isfinite(amax));  // FP32 overflow
        // FP32: threshold pivoting, the diagonal kept while it is at least a tenth of the
        // column's largest candidate
        if (sizeof(R) == 4 && fabs(A[k][k]) >= R(0.1) * amax) p = k;
        if (__any(p != k)) {
#pragma unroll
            for (int i = k + 1; i < KIN_N; ++i) {
                if (__any(p == i)) {
                    const bool sw = p == i;
#pragma unroll
                    for (int j = k; j < KIN_N; ++j) {
                        const R rk = A[k][j], ri = A[i][j];
                        A[k][j] = sw ? ri : rk;
                        A[i][j] = sw ? rk : ri;
                    }
                    const R rk = b[k], ri = b[i];
                    b[k] = sw ? ri : rk;
                    b[i] = sw ? rk : ri;
                }
            }
        }
        const R inv = R(1) / A[k][k];
        A[k][k] = inv;
#pragma unroll
        for (int i = k + 1; i < KIN_N; ++i) {
            const R l = A[i][k] * inv;
#pragma unroll
            for (int j = k + 1; j < KIN_N; ++j) A[i][j] = fma(-l, A[k][j], A[i][j]);
            b[i] = fma(-l, b[k], b[i]);
        }
    }
#pragma unroll
    for (int i = KIN_N - 1; i >= 0; --i) {
        R s = b[i];
#pragma unroll
        for (int j = i + 1; j < KIN_N; ++j) s = fma(-A[i][j], b[j], s);
        b[i] = s * A[i][i];
    }
    return ok;
}

// Outcome of one Newton iteration of a lane.
enum { KIN_CONTINUE = 0, KIN_ACCEPTED = 1, KIN_ATTEMPT_FAILED = 2 };

// One Newton iteration on the backward-Euler system of sub-step size h started from x
// (component i at x[64 i], the lane's LDS row): updates the iterate xk.  F32: the Newton matrix and right-hand side are rounded to FP32,
// factored with threshold pivoting and solved in FP32; the correction is promoted back to FP64
// (residual, rates and exponentials stay FP64).  On convergence the iterate is checked
// for negative mass fractions and its temperature is reset to the root of e(Y, T) = e0.
template <bool F32>
__device__ __forceinline__ int kin_newton_iteration(const KinLaneArgs &a, const double rho,
                                                    const double e0, const double *x,
                                                    double (&xk)[KIN_N], const double h, double &r_prev)
{
    double f[KIN_N];
    double A[KIN_N][KIN_N];
    kin_eval(kin_launder(a.K), rho, xk, f, A);
    double b[KIN_N];
    // chk stays 0 exactly when every entry is finite (0 times an infinity or a NaN is a NaN)
    double chk = 0.0;
#pragma unroll
    for (int i = 0; i < KIN_N; ++i) {
        b[i] = -((xk[i] - x[64 * i]) - h * f[i]);
        chk = fma(0.0, b[i], chk);
#pragma unroll
        for (int j = 0; j < KIN_N; ++j) {
            A[i][j] = (i == j ? 1.0 : 0.0) - h * A[i][j];
            chk = fma(0.0, A[i][j], chk);
        }
    }
    if (!(chk == 0.0)) return KIN_ATTEMPT_FAILED;  // some entry of A or G is not finite
    // The system is solved with the unknowns in the order (T, Y_1..Y_Ns): the temperature
    // row, whose entries are the largest, is then the first pivot row instead of being
    // exchanged upwards through the first columns, and most wavefronts skip the exchange
    // selects in more columns.  The order is a compile-time renaming of registers; the
    // solution is the same, up to rounding.
    double P[KIN_N][KIN_N], q[KIN_N];
#pragma unroll
    for (int i = 0; i < KIN_N; ++i) {
        q[i] = b[KIN_VAR(i)];
#pragma unroll
        for (int j = 0; j < KIN_N; ++j) P[i][j] = A[KIN_VAR(i)][KIN_VAR(j)];
    }
    double d[KIN_N];
    if (F32) {
        float Af[KIN_N][KIN_N], bf[KIN_N];
#pragma unroll
        for (int i = 0; i < KIN_N; ++i) {
#pragma unroll
            for (int j = 0; j < KIN_N; ++j) Af[i][j] = (float)P[i][j];
            bf[i] = (float)q[i];
        }
        if (!kin_lu_solve<float>(Af, bf)) return KIN_ATTEMPT_FAILED;
#pragma unroll
        for (int i = 0; i < KIN_N; ++i) d[KIN_VAR(i)] = (double)bf[i];
    } else {
        if (!kin_lu_solve<double>(P, q)) return KIN_ATTEMPT_FAILED;
#pragma unroll
        for (int i = 0; i < KIN_N; ++i) d[KIN_VAR(i)] = q[i];
    }
    bool conv = true;
    double chk2 = 0.0;
#pragma unroll
    for (int i = 0; i < KIN_N; ++i) {
        xk[i] += d[i];
        chk2 += xk[i] - xk[i];
        const double atol = (i < KIN_NS) ? a.atol_Y : a.atol_T;
        conv = conv && (fabs(d[i]) <= atol + a.rtol * fabs(xk[i]));
    }
    if (!(chk2 == 0.0)) return KIN_ATTEMPT_FAILED;
    if (xk[KIN_NS] < KIN_T_MIN || xk[KIN_NS] > KIN_T_MAX) return KIN_ATTEMPT_FAILED;
    if (!conv && !a.point_implicit) {
        // weighted norm of this update; growth by more than diverge_ratio over the previous
        // update abandons the attempt (Newton diverging)
        if (a.diverge_ratio > 0.0) {
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < KIN_N; ++i) {
                const double atol = (i < KIN_NS) ? a.atol_Y : a.atol_T;
                r = fmax(r, fabs(d[i]) / (atol + a.rtol * fabs(xk[i])));
            }
            if (r_prev >= 0.0 && r > a.diverge_ratio * r_prev) return KIN_ATTEMPT_FAILED;
            r_prev = r;
        }
        return KIN_CONTINUE;
    }
    bool neg = false;
#pragma unroll
    for (int s = 0; s < KIN_NS; ++s) neg = neg || (xk[s] < -a.y_neg);
    if (neg && !a.point_implicit) return KIN_ATTEMPT_FAILED;
    double T;
    if (!kin_invert_T(a.K, xk, e0, xk[KIN_NS], T)) return KIN_ATTEMPT_FAILED;
    xk[KIN_NS] = T;
    return KIN_ACCEPTED;
}

// Persistent lanes.  Every loop trip performs one Newton iteration for the cell each lane
// holds, so lanes whose cells need many iterations (sub-step halving) do not hold back the
// rest of their wavefront: a lane that finishes its cell stores it and takes the next cell.
//
// Cells reach the lanes through a per-wavefront queue in LDS: the wavefront claims KIN_QCHUNK
// consecutive launch positions with one atomic, and its 64 lanes load those cells' states into
// the queue together; lanes that need a cell then read a queue slot.  One claim and one load
// round trip serve 64 refills, and the cache lines of neighbouring cells are read and written
// by one wavefront, through one L2, instead of by whichever wavefronts of the device refilled
// at that moment.
//
// Sub-stepping is dyadic, time counted in ticks of dt 2^-Lc so that every sub-step boundary
// is exact.  Adaptive (L_forced < 0): start at h = dt, halve on a failed attempt and retry
// from the last accepted state, double after an accepted sub-step that ends on a boundary of
// the doubled step; a level beyond L_max or more than max_iters Newton iterations fail the
// cell, which keeps its input state.  Replay (L_forced >= 0): 2^L_forced equal sub-steps.
#define KIN_QCHUNK 64
#define KIN_QV (KIN_N + 3)   // queued doubles per cell: rho, e0, dt, then Y_1..Y_Ns, T
#define KIN_QI 4             // queued integers per cell: arena base, span cells, cell, launch cell

template <bool F32>
__device__ __forceinline__ void kin_lane_run(const KinLaneArgs &a)
{
    __shared__ double kin_qv[KIN_BLOCK / 64][KIN_QV][KIN_QCHUNK];
    __shared__ long long kin_qi[KIN_BLOCK / 64][KIN_QI][KIN_QCHUNK];
    // each lane's sub-step start state x (component s at x[64 s]): kept in LDS, where it is
    // read once per Newton iteration, instead of in registers through the whole iteration
    __shared__ double kin_xs[KIN_BLOCK / 64][KIN_N][64];
    const int lane = (int)(threadIdx.x & 63u);
    const int wv = (int)(threadIdx.x >> 6);
    const bool adapt = a.L_forced < 0;
    const int Lc = adapt ? a.L_max : a.L_forced;
    const unsigned long long end = 1ull << Lc;

    long long i = -1;    // cell index within the lane's span
    char *base = nullptr;
    long long nspan_cells = 0;
    double dt = 0.0;
    bool need = true;    // the lane has no cell in progress
    bool done = false;   // no cell is left for the lane
    int qn = 0, qh = 0;  // valid slots of the wavefront's queue, next slot to hand out
    bool qend = false;   // the counter ran past the last cell
    double rho = 0.0, e0 = 0.0;
    double xk[KIN_N];
    double *const x = &kin_xs[wv][0][lane];
#pragma unroll
    for (int s = 0; s < KIN_N; ++s) xk[s] = 0.0;
    unsigned long long t = 0, hsh = KIN_SCHED_SEED;
    int l = 0, k = 0, iters = 0, level = 0;
    bool failed = false;
    double r_prev = -1.0;  // weighted norm of the previous update of the current attempt
#ifdef KIN_TRACE
    unsigned long long *tr = nullptr;  // this cell's schedule record
#endif

    for (;;) {
        // ---- hand queued cells to lanes that need one, refilling the queue ---------------------
        // Take the cell in queue slot q: its state to registers, or, for an invalid input,
        // status 3 written at once (the lane then still needs a cell).
        auto take = [&](const int q) {
            base = (char *)kin_qi[wv][0][q];
            nspan_cells = kin_qi[wv][1][q];
            i = kin_qi[wv][2][q];
#ifdef KIN_TRACE
            tr = a.trace + (size_t)kin_qi[wv][3][q] * a.trace_words;
            tr[0] = 0;
#endif
            need = false;
            rho = kin_qv[wv][0][q];
            e0 = kin_qv[wv][1][q];
            dt = kin_qv[wv][2][q];
#pragma unroll
            for (int s = 0; s < KIN_N; ++s) xk[s] = kin_qv[wv][3 + s][q];
            double chk = rho - rho + e0 - e0 + dt - dt;
#pragma unroll
            for (int s = 0; s < KIN_N; ++s) chk += xk[s] - xk[s];
            if (!(chk == 0.0) || !(rho > 0.0) || !(dt >= 0.0) || xk[KIN_NS] < KIN_T_MIN ||
                xk[KIN_NS] > KIN_T_MAX) {
                kin_stat(base, nspan_cells, 0)[i] = 3;
                kin_stat(base, nspan_cells, 1)[i] = 0;
                kin_stat(base, nspan_cells, 2)[i] = 0;
                kin_sched(base, nspan_cells)[i] = KIN_SCHED_SEED;
                need = true;
            } else {
#pragma unroll
                for (int s = 0; s < KIN_N; ++s) x[64 * s] = xk[s];
                t = 0;
                l = adapt ? 0 : a.L_forced;
                level = l;
                k = 0;
                iters = 0;
                failed = false;
                hsh = KIN_SCHED_SEED;
            }
        };
        const unsigned long long want = __ballot(need && !done);
        if (want) {
            const int cnt = __popcll(want);
            const unsigned int lo = (unsigned int)want, hi = (unsigned int)(want >> 32);
            const int rank = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            const bool wants = need && !done;
            // first from what is left in the queue (read before the queue is refilled) ...
            const int take1 = min(cnt, qn - qh);
            if (wants && rank < take1) take(qh + rank);
            qh += take1;
            // ... then from a freshly claimed chunk
            if (cnt > take1 && !qend) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                unsigned long long g0 = 0;
                if (lane == 0) g0 = atomicAdd(a.counter, (unsigned long long)KIN_QCHUNK);
                g0 = __shfl(g0, 0);
                const long long left = a.total - (long long)g0;
                qn = left <= 0 ? 0 : (left < KIN_QCHUNK ? (int)left : KIN_QCHUNK);
                qh = 0;
                qend = qn == 0;
                if (lane < qn) {
                    const unsigned long long gi = g0 + (unsigned long long)lane;
                    int j = 0;
                    while (j + 1 < a.nspan && (unsigned long long)a.span[j + 1].start <= gi) ++j;
                    char *b = a.span[j].base;
                    const long long n = a.span[j].n;
                    long long c = (long long)gi - a.span[j].start;
                    if (a.span[j].order) {
                        const long long o = a.span[j].order[c];
                        if ((unsigned long long)o < (unsigned long long)n) c = o;
                    }
                    const double *Yin = kin_Y(b, n);
                    kin_qv[wv][0][lane] = kin_rho(b, n)[c];
                    kin_qv[wv][1][lane] = kin_e0(b, n)[c];
                    kin_qv[wv][2][lane] = a.span[j].dt;
#pragma unroll
                    for (int s = 0; s < KIN_NS; ++s) kin_qv[wv][3 + s][lane] = Yin[s * n + c];
                    kin_qv[wv][3 + KIN_NS][lane] = kin_T(b, n)[c];
                    kin_qi[wv][0][lane] = (long long)b;
                    kin_qi[wv][1][lane] = n;
                    kin_qi[wv][2][lane] = c;
                    kin_qi[wv][3][lane] = a.span[j].start + c;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int take2 = min(cnt - take1, qn);
                if (wants && rank >= take1 && rank - take1 < take2) take(rank - take1);
                qh = take2;
            }
            if (wants && need && qend && qh >= qn) {
                done = true;
                i = -1;
            }
        }
        if (!__any(!need)) {
            if (!__any(!done)) break;   // every lane has run out of cells
            continue;                   // only refills (bad inputs) this trip
        }
        if (!need) {
            int outcome;
            int st = -1;  // >= 0: the cell is finished with this status
            if (k == 0 && iters >= a.max_iters) {
                st = 2;
                outcome = KIN_CONTINUE;
            } else {
                ++iters;
                if (k == 0) r_prev = -1.0;
                outcome = kin_newton_iteration<F32>(a, rho, e0, x, xk, ldexp(dt, -l), r_prev);
                if (outcome == KIN_CONTINUE && ++k >= a.k_max) outcome = KIN_ATTEMPT_FAILED;
            }
            if (outcome != KIN_CONTINUE)
                hsh = (hsh ^ (unsigned long long)(2 * l + (outcome == KIN_ACCEPTED))) * KIN_SCHED_PRIME;
#ifdef KIN_TRACE
            if (outcome != KIN_CONTINUE) {
                const unsigned long long na = tr[0];
                if (na < 64ull * (unsigned long long)(a.trace_words - 1)) {
                    const unsigned long long bit = (unsigned long long)(outcome == KIN_ACCEPTED) << (na & 63);
                    tr[1 + (na >> 6)] = ((na & 63) ? tr[1 + (na >> 6)] : 0ull) | bit;
                }
                tr[0] = na + 1;
            }
#endif
            if (outcome == KIN_ACCEPTED) {
#pragma unroll
                for (int s = 0; s < KIN_N; ++s) x[64 * s] = xk[s];
                t += 1ull << (Lc - l);
                if (adapt && l > 0 && (t & ((1ull << (Lc - l + 1)) - 1ull)) == 0ull) --l;
                k = 0;
                if (t >= end) st = failed ? 1 : 0;
            } else if (outcome == KIN_ATTEMPT_FAILED) {
#pragma unroll
                for (int s = 0; s < KIN_N; ++s) xk[s] = x[64 * s];
                k = 0;
                if (!adapt) {
                    st = 2;
                } else {
                    failed = true;
                    ++l;
                    if (l > level) level = l;
                    if (l > a.L_max) { level = a.L_max; st = 2; }
                }
            }
            if (st >= 0) {
                if (st != 2) {
                    double *Yout = kin_Y(base, nspan_cells);
#pragma unroll
                    for (int s = 0; s < KIN_NS; ++s) Yout[s * nspan_cells + i] = x[64 * s];
                    kin_T(base, nspan_cells)[i] = x[64 * KIN_NS];
                }
                kin_stat(base, nspan_cells, 0)[i] = st;
                kin_stat(base, nspan_cells, 1)[i] = level;
                kin_stat(base, nspan_cells, 2)[i] = iters;
                kin_sched(base, nspan_cells)[i] = hsh;
                need = true;
            }
        }
    }
}

extern "C" __global__ void __launch_bounds__(KIN_BLOCK) kin_lane_f64(KinLaneArgs a)
{
    kin_lane_run<false>(a);
}

// Cost class of each cell of span 0 for a first advance (no iteration counts yet): the octave
// of the relative temperature change that the source term predicts over dt, |dT/dt| dt / T,
// clamped to 0..7 (7: a change of T itself or more; 0: below T / 128).  Cells whose
// temperature moves fastest take the most sub-steps.  The class only orders the cells.
extern "C" __global__ void __launch_bounds__(KIN_BLOCK) kin_lane_cost(KinLaneArgs a, int *key)
{
    const long long i = (long long)blockIdx.x * KIN_BLOCK + threadIdx.x;
    const long long n = a.span[0].n;
    if (i >= n) return;
    char *base = a.span[0].base;
    const double *Yin = kin_Y(base, n);
    double x[KIN_N];
#pragma unroll
    for (int s = 0; s < KIN_NS; ++s) x[s] = Yin[s * n + i];
    x[KIN_NS] = kin_T(base, n)[i];
    const double rho = kin_rho(base, n)[i];
    const double dt = a.span[0].dt;
    bool ok = rho > 0.0 && x[KIN_NS] >= KIN_T_MIN && x[KIN_NS] <= KIN_T_MAX;
#pragma unroll
    for (int s = 0; s < KIN_N; ++s) ok = ok && __builtin_isfinite(x[s]);
    int c = 0;
    if (ok) {
        double f[KIN_N], J[KIN_N][KIN_N];
        kin_eval(kin_launder(a.K), rho, x, f, J);
        const double p = fabs(f[KIN_NS]) * dt / x[KIN_NS];
        if (!(p < 1.0)) c = 7;
        else if (p > 0.0) c = max((int)floor(log2(p)) + 7, 0);
    }
    key[i] = c;
}

extern "C" __global__ void __launch_bounds__(KIN_BLOCK) kin_lane_f32lu(KinLaneArgs a)
{
    kin_lane_run<true>(a);
}
