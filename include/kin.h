/*
 * kin.h -- C ABI of libkin, the MI355X (gfx950) implicit chemical-kinetics library.
 *
 * The library advances batches of independent cells, each a constant-density,
 * constant-internal-energy 0-D reactor, over one time step dt by Newton-iterated backward
 * Euler with dyadic sub-step halving.  This is the chemistry half of the operator-split
 * reactive Euler solver of Le & Cambier (arXiv:1110.4903): the operator split itself
 * (Sec. 2, Eq. "operator_splitting") hands the chemistry one sub-step per flow step, each
 * cell is independent (Sec. 4.2), and the per-cell work is the point-implicit system
 * (I - dt dOmega/dQ) dQ = dt Omega of Sec. 3.2 (Eq. "kinetics") with rates built from the
 * Arrhenius law, the equilibrium constant and third-body sums of Sec. 3.2.
 *
 * Conventions
 *   - Plain C types only; every pointer is either host memory or device memory as stated.
 *   - Units at the boundary are SI: rho kg/m^3, T K, e J/kg, dt s.  Mechanism data are in
 *     the usual CGS kinetics units (mol, cm^3, s) and NASA-7 dimensionless coefficients.
 *   - Cell arrays are structure-of-arrays: rho[n], T[n], e0[n], and Y species-major
 *     [Ns][n] (cell index fastest), which is also the layout kept in device memory.
 *   - Every call returns a kin_status; KIN_OK is 0.  The message of the calling thread's
 *     last failure is available from kin_last_error().  No C++ exception crosses the ABI.
 *   - A per-cell numerical failure is not a call error: it is reported in the cell's status.
 *   - Thread safety: a context is guarded by an internal mutex; calls on one context from
 *     several host threads are serialised.  Work is enqueued on the caller's HIP stream.
 *   - KIN_EDEVICE means a HIP runtime error; the context must then be destroyed.
 */
#ifndef KIN_H
#define KIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KIN_OK = 0,
    KIN_EINVAL = 1,     /* invalid argument or mechanism */
    KIN_ENOMEM = 2,     /* the request exceeds the context's device-memory budget */
    KIN_EBUSY = 3,      /* the object is still referenced */
    KIN_ENOTFOUND = 4,  /* unknown mechanism or instance id */
    KIN_EDEVICE = 5,    /* HIP runtime failure; destroy the context */
    KIN_ECOMPILE = 6    /* run-time compilation of a mechanism kernel failed */
} kin_status;

typedef enum { KIN_FP64 = 0, KIN_FP32_LU = 1 } kin_precision;
/* Where caller buffers live.  KIN_MEM_HOST: pageable host memory, copied synchronously.
 * KIN_MEM_DEVICE: device memory, copied in stream order.  KIN_MEM_PINNED: page-locked host
 * memory (hipHostMalloc), copied in stream order without waiting; the caller keeps the buffer
 * alive and unchanged until the stream has passed the copy. */
typedef enum { KIN_MEM_HOST = 0, KIN_MEM_DEVICE = 1, KIN_MEM_PINNED = 2 } kin_mem;

/* Kernel layouts: one cell per lane with the Newton matrix in registers (ns <= 15), one cell
 * per 64-wide wavefront with one matrix row per lane and the Jacobian staged in LDS
 * (ns <= 63), or one cell per wavefront with the cell's whole matrix in global memory, which
 * is what the paper's first kinetics kernel keeps there (Sec. 4.2; any ns up to 255, the
 * automatic choice above 63).  The global layout allocates its workspace (at most 16 GiB)
 * stream-ordered on the launch stream, or with the graph of a batched advance, and is bound
 * by HBM bandwidth. */
typedef enum { KIN_LAYOUT_AUTO = 0, KIN_LAYOUT_LANE = 1, KIN_LAYOUT_WAVE = 2, KIN_LAYOUT_GLOBAL = 3 } kin_layout;

/* Per-cell status codes written by kin_advance. */
enum {
    KIN_CELL_OK = 0,         /* accepted as one sub-step of dt */
    KIN_CELL_OK_HALVED = 1,  /* accepted after at least one sub-step halving */
    KIN_CELL_FAILED = 2,     /* halving passed L_max; the cell keeps its input state */
    KIN_CELL_BAD_INPUT = 3   /* non-finite input, rho <= 0 or T outside [200, 6000] K */
};

typedef struct kin_ctx kin_ctx;

typedef struct {
    int32_t device;          /* HIP device ordinal */
    uint64_t hbm_budget;     /* bytes of instance state the context may hold; 0 = no limit.
                              * A budget is reserved at creation as one device pool that
                              * instances are carved from first-fit (no hipMalloc or hipFree
                              * per instance); an upload that finds no free block of its
                              * footprint fails with KIN_ENOMEM. */
    const char *tune_cache;  /* autotuner cache file (JSON); NULL = $KIN_TUNE_CACHE or none */
    uint32_t flags;          /* KIN_CTX_* bits, 0 = none */
} kin_ctx_opts;

/* kin_ctx_opts.flags: record a pair of events on the launch stream right around the advance
 * kernel of every single-instance kin_advance, for kin_kernel_times. */
enum { KIN_CTX_TIME_KERNELS = 1 };

/* Mechanism description (host memory, copied by kin_mech_upload; the caller keeps it).
 * Reactions have up to three reactant and three product entries (index, coefficient);
 * unused entries have index -1.  A reaction with tb[r] >= 0 multiplies its net rate by the
 * third-body concentration sum_s eff[tb[r]][s] X_s (Sec. 3.2, rate-of-progress equation). */
typedef struct {
    int32_t ns;                /* species, 1..255 (over 63: the global-memory layout only) */
    int32_t ne;                /* elements, >= 1 */
    int32_t nr;                /* reactions, >= 1 */
    int32_t ntb;               /* rows of eff */
    const double *M;           /* [ns] molar mass, g/mol */
    const int8_t *elem;        /* [ns][ne] atoms of each element */
    const double *nasa;        /* [ns][2][7]: set 0 for T < T_mid, set 1 otherwise */
    const double *T_mid;       /* [ns] K */
    const int32_t *reac_idx;   /* [nr][3] */
    const int32_t *reac_nu;    /* [nr][3], 1..3 where used */
    const int32_t *prod_idx;   /* [nr][3] */
    const int32_t *prod_nu;    /* [nr][3] */
    const double *A;           /* [nr] pre-exponential factor, CGS units, > 0 */
    const double *b;           /* [nr] temperature exponent */
    const double *Ta;          /* [nr] activation temperature E/R, K */
    const int32_t *reversible; /* [nr] 1: reverse rate from the equilibrium constant; 0: none */
    const int32_t *tb;         /* [nr] -1 or row of eff */
    const double *eff;         /* [ntb][ns] third-body efficiencies, >= 0 */
} kin_mech_desc;

/* Newton / sub-stepping controls.  Defaults (kin_default_solver_opts): rtol 1e-12,
 * atol_Y 1e-20, atol_T 1e-9 K, y_neg 1e-10, k_max 10, L_max 40, layout AUTO, L_forced -1,
 * max_iters 100000, point_implicit 0, diverge_ratio 2. */
typedef struct {
    double rtol;       /* Newton converged when |dx_i| <= atol_i + rtol |x_i| for all i */
    double atol_Y;
    double atol_T;
    double y_neg;      /* a converged iterate with some Y_s < -y_neg is rejected */
    int32_t k_max;     /* Newton iterations per sub-step attempt */
    int32_t L_max;     /* deepest halving level, sub-step dt 2^-L, 0..62 */
    int32_t layout;    /* kin_layout */
    int32_t L_forced;  /* -1: adaptive; >= 0: exactly 2^L_forced equal sub-steps */
    int32_t max_iters; /* Newton iterations per cell before it is declared FAILED */
    int32_t point_implicit; /* 1: the paper's point-implicit step (Sec. 3.2, Eq. "kinetics"):
                             * one linearised backward-Euler step over the whole dt,
                             * (I - dt J(x_n)) dx = dt f(x_n), taken without a convergence test
                             * or a negative-Y check, followed by the temperature inversion.
                             * k_max, L_max and L_forced are then ignored; a failure
                             * (non-finite, zero pivot, T out of range) gives status 2.
                             * FP64 only: without Newton's refinement an FP32 factorisation
                             * of I - dt J carries its full rounding error into the result,
                             * so kin_advance rejects it with KIN_EINVAL for KIN_FP32_LU. */
    double diverge_ratio;   /* an attempt fails early when an update's weighted norm
                             * max_i |dx_i| / (atol_i + rtol |x_i|) exceeds diverge_ratio
                             * times the previous iteration's (Newton diverging); 0 disables */
} kin_solver_opts;

/* Fill s with the defaults above.
 * Paper: Sec. 3.2, Eq. "kinetics" (the implicit system these controls iterate); the
 * constants themselves are this library's readings, the paper gives none. */
void kin_default_solver_opts(kin_solver_opts *s);

/* Message of the calling thread's last non-OK status ("" if none).
 * Paper: no passage (error reporting of this library). */
const char *kin_last_error(void);

/* Create a context on a device.  o may be NULL (device 0, no budget, no tune cache).
 * Paper: Sec. 5.2, the device memory that bounds how many cells' Jacobians are held at once,
 * which the optional budget caps. */
kin_status kin_create(kin_ctx **out, const kin_ctx_opts *o);

/* Free every device allocation and compiled module of the context.  Safe on NULL.
 * Paper: no passage (resource release). */
void kin_destroy(kin_ctx *ctx);

/* Validate and copy a mechanism to the device; returns its id.  Validation: counts in
 * range, indices in range, coefficients 1..3, every reaction element-balanced, A > 0,
 * finite parameters, cp > 0 over [200, 6000] K, efficiencies >= 0.  Species count decides
 * the default layout (lane layout when ns <= 15); a mechanism that will run the lane
 * layout gets its kernels compiled here (hipRTC, gfx950).
 * Paper: Sec. 3.2, where species data and elementary reactions are read from data files
 * separate from the solver; the reaction form, Arrhenius law, equilibrium constant and
 * third-body sum that the tables parameterise are the equations of Sec. 3.2. */
kin_status kin_mech_upload(kin_ctx *ctx, const kin_mech_desc *d, int32_t *mech_id);

/* Release a mechanism's device tables and kernels.  KIN_EBUSY while instances still use it.
 * Paper: Sec. 3.2 (the mechanism data uploaded by kin_mech_upload). */
kin_status kin_mech_release(kin_ctx *ctx, int32_t mech_id);

/* Copy n_cells cell states into a new device-resident instance of a mechanism.  rho, T,
 * Y (and e0) live in host or device memory as `where` says; device copies are enqueued on
 * `stream` (a hipStream_t, NULL = the null stream), host copies complete before return.
 * e0_or_null: per-cell internal energy e0 (J/kg) the step conserves; NULL computes
 * e0 = e(Y, T) on the device.  KIN_ENOMEM if the context budget would be exceeded.
 * Paper: Sec. 4.2, each cell's kinetics is independent of every other cell's, so cells are
 * stored as independent structure-of-arrays records; Sec. 2, Eq. energy, for e0. */
kin_status kin_state_upload(kin_ctx *ctx, int32_t mech_id, int64_t n_cells, const double *rho,
                            const double *T, const double *Y, const double *e0_or_null,
                            kin_mem where, void *stream, int32_t *inst_id);

/* Overwrite an existing instance's state (same cell count) without allocating.
 * Paper: Sec. 4.2 (independent cells), as kin_state_upload. */
kin_status kin_state_reset(kin_ctx *ctx, int32_t inst_id, const double *rho, const double *T,
                           const double *Y, const double *e0_or_null, kin_mem where,
                           void *stream);

/* Advance n instances by their dts[n] on `stream`, asynchronously.  Each instance's T and Y
 * are replaced by the step's result (a failed cell keeps its state) and its status, level
 * (deepest halving level) and iters (Newton iterations including failed tries) are written.
 * s may be NULL for the defaults.  With n > 1 all instances go out in one graph launch.
 * A single instance of at least 262144 cells in the lane layout, or 32768 in the others
 * (about four times the cells a layout keeps in flight), takes its cells in cost order.  When
 * its iters come from an advance of its current state (no kin_state_reset or conserved
 * reset since), the classes are the iterations each cell needed: 320 or more first, then
 * 160-319, 80-159, 40-79, 20-39, 10-19, 5-9 and the rest.  Otherwise, in the lane layout,
 * they are the octave of the temperature change the source term predicts over dt.  Each class
 * keeps index order.  This shortens the launch's tail; every cell's result is bitwise the
 * same in any order.  Advances of one instance must be ordered on one stream (or
 * synchronised), as the order is computed on `stream` from the previous advance's iters.
 * Paper: Sec. 3.2, Eq. "kinetics", solved by Gaussian elimination per cell; Sec. 4.2, one
 * independent system per cell; iteration and halving are this library's additions. */
kin_status kin_advance(kin_ctx *ctx, const int32_t *inst_ids, const double *dts, int32_t n,
                       kin_precision prec, const kin_solver_opts *s, void *stream);

/* kin_advance of one instance that also records every cell's sub-step schedule, for checking
 * a result against a reference that follows the same sub-steps.  trace: device memory of
 * n_cells * words uint64 (caller-owned, words 2..4096); cell i's record is trace[i * words ..]:
 * word 0 the number of sub-step attempts, words 1.. their outcomes, attempt j accepted iff bit
 * j % 64 of word 1 + j / 64 is set (the first 64 (words - 1) attempts are recorded; the count
 * is always complete).  The sub-step sizes follow from the outcomes: a rejection retries the
 * same start at the next level, an acceptance at level l advances by dt 2^-l and drops a level
 * when the elapsed time is aligned to the coarser grid.  The cells' arithmetic, results and
 * diagnostics are those of kin_advance (cells taken in index order); the lane layout runs a
 * separately compiled build of its kernels with the recorder.  Enqueued on `stream`.
 * Paper: Sec. 3.2, Eq. "kinetics" (the sub-steps over which it is solved). */
kin_status kin_advance_trace(kin_ctx *ctx, int32_t inst_id, double dt, kin_precision prec,
                             const kin_solver_opts *s, int32_t words, uint64_t *trace, void *stream);

/* kin_advance without any device allocation, for callers that cannot allocate: code under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc.  Same arguments, checks,
 * per-cell results and diagnostics as kin_advance, bitwise.  The launches (instances grouped
 * by mechanism and layout, at most 64 per launch) go out one after another on `stream`, in
 * index order (no cost order, no internal graph or streams).  Their work counters and the
 * matrices of global-layout launches live in a fixed 256 MiB array of device memory that each
 * device holds from the library's first context on it until the process ends; a global-layout
 * launch keeps as many cells in flight as that array has matrix slots for, which bounds its
 * parallelism, not its size.  Limits: at most 64 instances per call (KIN_EINVAL beyond).
 * Lane-layout kernels must already be compiled for the block size in use (kin_mech_upload does
 * so for the default, kin_set_layout for another); otherwise KIN_EINVAL.  All calls on one
 * device share that array: two calls whose work overlaps on the device (different streams, or
 * different contexts or host threads, not ordered by the caller) race on it and give undefined
 * results.  Calls ordered on one stream are safe.
 * Paper: no passage; the callers are those that cannot allocate (the computation is that of
 * kin_advance). */
kin_status kin_advance_noalloc(kin_ctx *ctx, const int32_t *inst_ids, const double *dts, int32_t n,
                               kin_precision prec, const kin_solver_opts *s, void *stream);

/* Copy an instance's state (T[n], Y[Ns][n]), the conserved internal energy e0[n] and the
 * per-cell diagnostics of the last advance into caller buffers; any pointer may be NULL.
 * Re-uploading T, Y with this e0 resumes the run bitwise (checkpoint / restart).
 * Host destinations: synchronous.  Device destinations: enqueued on `stream`.
 * Paper: Sec. 4.2 (independent per-cell results of the system of Sec. 3.2, Eq. "kinetics"). */
kin_status kin_download(kin_ctx *ctx, int32_t inst_id, double *T, double *Y, double *e0,
                        int32_t *status, int32_t *level, int32_t *iters, kin_mem where,
                        void *stream);

/* Per-cell sub-step schedule of the last advance: a 64-bit FNV-1a hash of the sequence of
 * sub-step attempts, starting from 0xcbf29ce484222325 and folding in, per attempt at level l,
 * h = (h ^ (2 l + accepted)) * 0x100000001b3.  Two runs whose hashes agree took the same
 * sub-steps, so their results differ only by arithmetic, not by the step sizes taken.
 * Paper: Sec. 3.2, Eq. "kinetics" (the sub-steps over which it is solved; halving itself is
 * this library's addition). */
kin_status kin_download_schedule(kin_ctx *ctx, int32_t inst_id, uint64_t *sched, kin_mem where,
                                 void *stream);

/* Operator-split adapter (Sec. 2: the energy equation and the operator-splitting equation).
 * The fluid side of the split carries partial densities and an energy that leaves out the
 * species formation energies; the chemistry sub-step changes the partial densities and must
 * account for the change of formation energy in that energy.  Here the left-out part of each
 * species' internal energy is its value at T_ref = 298.15 K, e_s(T_ref) (J/kg, NASA-7 h with
 * the formation enthalpy), so the fluid-side energy is the sensible internal energy
 *     E_sens = sum_s rho_s (e_s(T) - e_s(T_ref))        (J/m^3, kinetic energy excluded).
 *
 * kin_state_upload_conserved creates an instance from rho_s [Ns][n] (kg/m^3, species-major)
 * and E_sens [n]: rho = sum_s rho_s, Y_s = rho_s / rho, e0 = E_sens / rho + sum_s Y_s
 * e_s(T_ref), and T the root of e(Y, T) = e0 in [200, 6000] K found by Newton from T_guess [n]
 * (NULL: 1500 K) with a bisection fallback; a cell without a root gets T = NaN, which the next
 * kin_advance reports as bad input.  All three arrays live where `where` says (host copies
 * complete before return); the conversion runs on the device on `stream`.  Errors as
 * kin_state_upload.
 * Paper: Sec. 2, Eq. energy (formation energies left out of E) and Eq. operator_splitting. */
kin_status kin_state_upload_conserved(kin_ctx *ctx, int32_t mech_id, int64_t n_cells,
                                      const double *rho_s, const double *E_sens,
                                      const double *T_guess, kin_mem where, void *stream,
                                      int32_t *inst_id);

/* The same conversion into an existing instance of the same cell count, without allocating.
 * Paper: Sec. 2, Eq. energy and Eq. operator_splitting, as kin_state_upload_conserved. */
kin_status kin_state_reset_conserved(kin_ctx *ctx, int32_t inst_id, const double *rho_s,
                                     const double *E_sens, const double *T_guess, kin_mem where,
                                     void *stream);

/* The inverse conversion of an instance's current state into caller buffers: rho_s [Ns][n] =
 * rho Y_s and E_sens [n] = rho (e0 - sum_s Y_s e_s(T_ref)).  Since kin_advance holds rho and e0,
 * E_sens after a step differs from E_sens before it by minus the change of formation energy,
 * sum_s (rho_s,before - rho_s,after) e_s(T_ref): the source term of the energy equation.
 * Device destinations: computed in place on `stream`.  Host or pinned destinations: through a
 * stream-ordered device staging buffer; host copies complete before return.
 * Paper: Sec. 2, Eq. energy (the source term carries the change of formation energy) and
 * Eq. operator_splitting. */
kin_status kin_download_conserved(kin_ctx *ctx, int32_t inst_id, double *rho_s, double *E_sens,
                                  kin_mem where, void *stream);

/* Durations (ms) of the advance kernels of the single-instance kin_advance calls made since
 * the previous call, in launch order, measured by events recorded on the launch stream around
 * each kernel (only with KIN_CTX_TIME_KERNELS; the work-counter clear and the ordering kernels
 * of a cost-ordered step are outside).  Waits for those kernels.  Writes up to cap values into
 * ms (may be NULL with cap 0), the number recorded into *count, and forgets them.
 * Paper: Sec. 5.2 (the kernel's performance measured on the device). */
kin_status kin_kernel_times(kin_ctx *ctx, double *ms, int32_t cap, int32_t *count);

/* Wait for `stream` (NULL = the null stream).
 * Paper: no passage (stream synchronisation). */
kin_status kin_sync(kin_ctx *ctx, void *stream);

/* A stream (default priority) whose kernels run only on compute units [cu_begin, cu_end) of
 * the context's device, for a serving loop that keeps some units free of long launches so
 * that short requests do not queue behind them.  *stream receives a hipStream_t the
 * caller passes to kin_advance etc. and releases with kin_stream_destroy.  KIN_EINVAL unless
 * 0 <= cu_begin < cu_end <= number of compute units.
 * Paper: Sec. 5.2, which processes the domain in segments large enough to fill the device;
 * this bounds the compute units a launch may occupy instead of its cells. */
kin_status kin_stream_create(kin_ctx *ctx, int32_t cu_begin, int32_t cu_end, void **stream);
/* Destroy a stream made by kin_stream_create.  Paper: Sec. 5.2, as kin_stream_create. */
kin_status kin_stream_destroy(kin_ctx *ctx, void *stream);

/* Free an instance.  Work already enqueued on it must have completed (with a budget pool the
 * memory goes straight back to the pool, without a device synchronisation).
 * Paper: Sec. 5.2 (segments of the domain held one after another within the device memory). */
kin_status kin_instance_release(kin_ctx *ctx, int32_t inst_id);

/* Device bytes an instance of n_cells cells of a mechanism occupies (admission by footprint).
 * Paper: Sec. 5.2, where the per-cell memory limits the cells processed at once and the domain
 * is split into segments that fit. */
kin_status kin_footprint(const kin_ctx *ctx, int32_t mech_id, int64_t n_cells,
                         kin_precision prec, uint64_t *bytes);

typedef enum {
    KIN_Q_BYTES_IN_USE = 0,   /* out: uint64 */
    KIN_Q_LAYOUT = 1,         /* arg: mech id; out: int32 kin_layout chosen */
    KIN_Q_BLOCK = 2,          /* arg: mech id; out: int32 threads per block of that layout */
    KIN_Q_NUM_CU = 3,         /* out: int32 */
    KIN_Q_DEVICE_PTRS = 4,    /* arg: instance id; out: 7 x uint64 rho, e0, T, Y, status, level, iters */
    KIN_Q_JIT_SECONDS = 5,    /* arg: mech id; out: double compile time of its lane kernels */
    KIN_Q_LARGEST_FREE = 6,   /* out: uint64 largest free block of the budget pool (0 without one) */
    KIN_Q_TUNED = 7           /* arg: mech id; out: int32[20], (layout, block) autotuned for
                               * precision p and size class c at [2 (5 p + c)], -1 where none */
} kin_query_what;

/* Report what kin_query_what names.  Paper: Sec. 5.2 (memory in use against the device's), and
 * Sec. 4.2 (the kernel layout chosen for a mechanism). */
kin_status kin_query(const kin_ctx *ctx, int32_t what, int64_t arg, void *out);

/* Set a mechanism's layout and block size for every launch: lane 64/128/256 threads (a block's
 * LDS, 512 (2 ns + 9) bytes per wavefront, must stay within 64 KiB: 256 threads up to ns = 11),
 * wave 1..4 wavefronts, global 64 threads per block.  KIN_EINVAL otherwise.  Drops the
 * autotuner's per-size choices.
 * Paper: Sec. 4.1, block size as a tuning parameter; Sec. 4.2, the choice between keeping the
 * Jacobian in global memory or in on-chip memory. */
kin_status kin_set_layout(kin_ctx *ctx, int32_t mech_id, int32_t layout, int32_t block);

/* Autotuner: time one advance of an existing instance with every admissible kernel layout
 * and block size of its mechanism (lane layout with 64, 128 or 256 threads per block when
 * ns <= 15, within 64 KiB of LDS per block; wave layout with 1, 2 or 4 wavefronts per block; the global layout above 63
 * species), and keep the fastest for launches of the instance's size class and this
 * precision.  Size classes of a launch's cell count (a batched advance counts all instances
 * of a mechanism together): below 4096, 16384, 65536, 262144, and the rest.  A launch of a
 * class and precision without a tuned entry uses the mechanism's layout (kin_set_layout, or
 * the default by species count); kin_set_layout drops the tuned entries.  Each choice is also
 * recorded in the context's tune cache file (JSON, keyed by a hash of the mechanism, the
 * precision, the size class and the device), from which kin_mech_upload applies it later.
 * Tune at the cell count the launches will have.  The instance's state is restored
 * afterwards.  Outputs may be NULL.
 * Paper: Sec. 4.1 (block size tuned by measurement) and Sec. 4.2 (global versus on-chip
 * memory for the Jacobian, chosen by measurement). */
kin_status kin_autotune(kin_ctx *ctx, int32_t mech_id, int32_t inst_id, double dt,
                        kin_precision prec, int32_t *layout, int32_t *block, double *best_ms);

/* ---- The fluid step and the operator-split step ---------------------------------------------
 * A fluid grid of nx x ny cells of one mechanism holds the conserved variables of Sec. 2,
 * Q = (rho_s [Ns], rho u, rho v, E), as device memory [Ns + 3][ny][nx] (x fastest; SI units:
 * kg/m^3, kg/(m^2 s), J/m^3), with E = sum_s rho_s e_s(T) + rho |u|^2 / 2 and each species'
 * energy without its formation energy, e_s(T) - e_s(298.15 K) from the NASA-7 data (Sec. 2,
 * Eq. energy; the same energy as the conserved-variable adapter above).  Pressure is Dalton's
 * law (Eq. dalton) and the sound speed that of the frozen mixture, c^2 = (c_p / c_v) P / rho.
 * Boundaries: KIN_BC_PERIODIC, or KIN_BC_OUTFLOW (zero-gradient) on all four sides. */
enum { KIN_BC_PERIODIC = 0, KIN_BC_OUTFLOW = 1 };

/* Create a fluid grid (spacings dx, dy in m) for a mechanism; the library allocates its state
 * and workspace (about 3 (Ns + 3) + 4 doubles per cell plus the face fluxes).  nx, ny >= 1, and
 * >= 3 for KIN_BC_PERIODIC (the six-cell stencil wraps once); KIN_EINVAL otherwise.
 * Paper: Sec. 4.1, the whole domain stored as one-dimensional arrays per variable. */
kin_status kin_fluid_create(kin_ctx *ctx, int32_t mech_id, int32_t nx, int32_t ny, double dx, double dy,
                            int32_t bc, int32_t *fluid_id);
/* Free a fluid grid.  Paper: no passage (resource release). */
kin_status kin_fluid_release(kin_ctx *ctx, int32_t fluid_id);
/* Copy Q [Ns + 3][ny][nx] in or out (host copies complete before return, device copies are
 * enqueued on `stream`).  Paper: Sec. 2 (the conserved variables) and Sec. 4.1 (their layout). */
kin_status kin_fluid_upload(kin_ctx *ctx, int32_t fluid_id, const double *Q, kin_mem where, void *stream);
/* Copy Q out, as kin_fluid_upload copies it in.  Paper: Sec. 2 and Sec. 4.1, as kin_fluid_upload. */
kin_status kin_fluid_download(kin_ctx *ctx, int32_t fluid_id, double *Q, kin_mem where, void *stream);
/* Largest stable step: cfl times min over cells of dx / (|u| + c) and dy / (|v| + c); waits for
 * `stream`.  0 if a cell has no valid state.  Paper: Sec. 3.1 (the explicit time integration
 * these bounds limit). */
kin_status kin_fluid_max_dt(kin_ctx *ctx, int32_t fluid_id, double cfl, double *dt, void *stream);
/* One convective step of dt (Sec. 3.1): dimensional splitting, an x sweep then a y sweep (the
 * reverse with y_first != 0; alternating the order from step to step is the caller's choice),
 * each sweep three stages of the third-order strong-stability-preserving Runge-Kutta scheme over
 * the flux difference of MP5 faces (Eq. mp5, limited by Eqs. mp and ump, on the primitive
 * variables rho_s, u_n, u_t, P) and the HLLE flux (Eq. fluxhlle, taken in its upwind form:
 * (b+ F_L - b- F_R) / (b+ - b-) + b+ b- / (b+ - b-) (Q_R - Q_L)).  Asynchronous on `stream`.
 * Paper: Sec. 3.1 (fluid dynamics) and Sec. 4.1 (one thread per cell or face). */
kin_status kin_fluid_step(kin_ctx *ctx, int32_t fluid_id, double dt, int32_t y_first, void *stream);
/* One operator-split step of dt (Sec. 2, Eq. operator_splitting): the convective step above,
 * then the chemistry sub-step of the same cells through the conserved-variable adapter
 * (kin_state_reset_conserved with the partial densities and E - rho |u|^2 / 2, kin_advance of
 * dt with prec and s, kin_download_conserved back; momentum and kinetic energy are unchanged by
 * the chemistry).  inst_id must be an instance of the fluid's mechanism with nx ny cells (its
 * state is overwritten; the Newton iteration counts of its previous advance, if current, order
 * this step's cells by cost, which changes no result).  Asynchronous on `stream`.
 * Paper: Sec. 2, Eq. operator_splitting, with Eq. energy for the formation-energy source. */
kin_status kin_split_step(kin_ctx *ctx, int32_t fluid_id, int32_t inst_id, double dt, int32_t y_first,
                          kin_precision prec, const kin_solver_opts *s, void *stream);

/* Generate the lane-layout source for a mechanism and compile it for gfx950 with hipRTC,
 * without a device, both as kin_advance runs them and with the schedule recorder of
 * kin_advance_trace.  log (may be NULL) receives up to log_len bytes of compiler output.
 * Paper: Sec. 3.2 (the mechanism from data files, here validated and compiled). */
kin_status kin_jit_check(const kin_mech_desc *d, char *log, size_t log_len);

#ifdef __cplusplus
}
#endif
#endif
