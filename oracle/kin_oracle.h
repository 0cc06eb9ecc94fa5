/*
 * kin_oracle.h -- plain FP64 CPU oracle for the per-cell implicit chemical-kinetics update
 * of Le & Cambier, "Development of a Flow Solver with Complex Kinetics on the Graphic
 * Processing Units" (arXiv:1110.4903).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark call this library.  It shares no code, header, table or constant with
 * the HIP library: it is an independent, slow, obviously-correct restatement of the method
 * used to check that library's results.
 *
 * What it computes (paper Sec. 3.2 "Chemical Kinetics" and Sec. 2):
 *   - Arrhenius forward rate constants (Sec. 3.2, forward-rate equation);
 *   - reverse rate constants through the equilibrium constant built from the standard
 *     Gibbs energy change (Sec. 3.2, equilibrium-constant equation), with NASA 7-coefficient
 *     polynomials for cp, h and s;
 *   - rates of progress with the third-body sum (Sec. 3.2, rate-of-progress equation) and
 *     species net production (Sec. 3.2, production equation);
 *   - the implicit system (I - dt dOmega/dQ) dQ = dt Omega (Sec. 3.2, Eq. "kinetics") taken
 *     as Newton iterations on backward Euler in x = (Y_1..Y_Ns, T) for a constant-density,
 *     constant-internal-energy cell (energy bookkeeping of Sec. 2, Eq. "energy"), solved by
 *     Gaussian elimination with partial pivoting (Sec. 3.2 / Sec. 4.2), with sub-step halving
 *     on failure and a temperature inversion e(Y, T) = e0 after every accepted sub-step.
 *
 * Units: boundary in SI (rho kg/m^3, e J/kg, T K); kinetics in CGS (mol, cm^3, s).
 * Layouts: Y is species-major [Ns][n_cells]; matrices are row-major.
 */
#ifndef KIN_ORACLE_H
#define KIN_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NS_MAX 255

typedef struct {
    int ns, nr, ntb;
    const double *M;        /* [ns] molar mass, g/mol */
    const double *nasa;     /* [ns][2][7]: range 0 for T < T_mid, range 1 otherwise */
    const double *T_mid;    /* [ns] K */
    const int *reac_idx;    /* [nr][3] species index, -1 = empty */
    const int *reac_nu;     /* [nr][3] stoichiometric coefficient */
    const int *prod_idx;    /* [nr][3] */
    const int *prod_nu;     /* [nr][3] */
    const double *A;        /* [nr] CGS pre-exponential factor */
    const double *b;        /* [nr] temperature exponent */
    const double *Ta;       /* [nr] activation temperature E/R, K */
    const int *reversible;  /* [nr] 1 = reversible */
    const int *tb;          /* [nr] -1 = no third body, else row of eff */
    const double *eff;      /* [ntb][ns] third-body efficiencies */
} orc_mech;

typedef struct {
    double rtol, atol_Y, atol_T;
    double y_neg;           /* a converged iterate with some Y_s < -y_neg is rejected */
    int k_max, L_max;
    int max_iters;          /* Newton iterations per cell before it is declared failed */
    double diverge_ratio;   /* an attempt fails when an update's weighted norm
                               max_i |dx_i| / (atol_i + rtol |x_i|) exceeds diverge_ratio times
                               the previous iteration's (Newton diverging); 0 disables */
    int point_implicit;     /* 1: the point-implicit step of Sec. 3.2 (Eq. "kinetics"): one
                               linearised backward-Euler step over the whole dt,
                               (I - dt J(x_n)) dx = dt f(x_n), accepted without a convergence
                               test or a negative-Y check, then the temperature inversion; a
                               failure (non-finite, zero pivot, T out of range) is final */
} orc_opts;

/* Per-cell status codes. */
enum { ORC_OK = 0, ORC_OK_HALVED = 1, ORC_FAILED = 2, ORC_BAD_INPUT = 3 };

void orc_default_opts(orc_opts *o);

/* NASA-7 species functions at T: cp/R, h/(RT), s/R, d(cp/R)/dT (arrays of length ns). */
void orc_species_thermo(const orc_mech *m, double T, double *cp_R, double *h_RT,
                        double *s_R, double *dcpR_dT);

/* Mixture specific internal energy e(Y,T) (J/kg) and c_v (J/kg/K). */
double orc_mix_energy(const orc_mech *m, const double *Y, double T);
double orc_mix_cv(const orc_mech *m, const double *Y, double T);

/* Rate constants, third-body concentration, forward/backward progress (without the
 * third-body factor), net progress q and net molar production wdot (mol/cm^3/s). */
void orc_rates(const orc_mech *m, double rho, const double *Y, double T,
               double *kf, double *kb, double *Mconc, double *qf, double *qb,
               double *q, double *wdot);

/* Right-hand side f = dx/dt of the constant-(rho, e) cell, x = (Y, T). */
void orc_rhs(const orc_mech *m, double rho, const double *x, double *f);

/* Analytic Jacobian J = df/dx, row-major (ns+1)x(ns+1). */
void orc_jacobian(const orc_mech *m, double rho, const double *x, double *J);

/* Central finite-difference Jacobian (diagnostic for the analytic one). */
void orc_jacobian_fd(const orc_mech *m, double rho, const double *x, double *J);

/* LU with partial pivoting (first row of largest |a_ik|), in place, row-major n x n.
 * piv[k] = row swapped with row k at step k.  Returns 0, or -1 on an exactly zero pivot. */
int orc_lu_factor(int n, double *A, int *piv);
void orc_lu_solve(int n, const double *LU, const int *piv, double *b);

/* Solve e(Y, T) = e0 for T, starting from T_start.  Returns 0 on success. */
int orc_invert_T(const orc_mech *m, const double *Y, double e0, double T_start, double *T_out);

/* One backward-Euler sub-step of size h from x (in/out).  Returns 0 on success.  x_be (may
 * be NULL) receives the converged Newton iterate before the temperature inversion. */
int orc_be_substep(const orc_mech *m, double rho, double e0, double *x, double h,
                   const orc_opts *o, int *iters, double *x_be);

/* One cell over dt.  L_forced < 0: adaptive dyadic sub-stepping (halve on failure, double
 * after a success when aligned); L_forced >= 0: exactly 2^L_forced equal sub-steps.
 * *level = deepest halving level used, *iters = Newton iterations including failed tries,
 * *sched = 64-bit FNV-1a hash of the sequence of (level, accepted) sub-step attempts. */
int orc_advance_cell(const orc_mech *m, double rho, double e0, double *T, double *Y,
                     long stride, double dt, const orc_opts *o, int L_forced,
                     int *level, int *iters, unsigned long long *sched);

/* Batch over cells (OpenMP over cells, nthreads <= 0 = runtime default).
 * T[n] and Y[ns][n] are updated in place; status/level/iters may be NULL. */
void orc_advance(const orc_mech *m, long n, const double *rho, const double *e0,
                 double *T, double *Y, double dt, const orc_opts *o, int L_forced,
                 int *status, int *level, int *iters, unsigned long long *sched, int nthreads);

/* Advance one cell along a given sub-step schedule instead of choosing it: attempt j of the
 * schedule (bit j % 64 of word j / 64 of bits[]) was accepted (1) or rejected (0) by another
 * implementation.  The sub-step sizes follow from those bits by the adaptive rule of
 * orc_advance_cell (a rejection retries the same start at level l + 1, an acceptance at level l
 * advances by dt 2^-l and drops a level when the elapsed time is aligned to the coarser grid).
 * A rejected attempt is skipped; an accepted one is the backward-Euler sub-step solved to
 * convergence from the last accepted state (Newton without the divergence test and with at
 * least 50 iterations, then the temperature inversion).  So the result is this oracle's
 * backward-Euler solution over exactly the other side's sub-steps.
 * Returns ORC_OK or ORC_OK_HALVED when the schedule covers dt, ORC_FAILED (state unchanged)
 * when it ends before dt (the other side failed the cell), ORC_BAD_INPUT on bad input, and -1
 * when an attempt the schedule accepts does not converge here (result undefined).
 * *level, *iters and *sched are as for orc_advance_cell (sched over the given schedule). */
int orc_follow_cell(const orc_mech *m, double rho, double e0, double *T, double *Y, long stride,
                    double dt, const orc_opts *o, const unsigned long long *bits, long count,
                    int *level, int *iters, unsigned long long *sched);

/* Batch form: trace[n][words], word 0 of a cell the number of attempts, words 1.. their bits
 * (a cell whose count exceeds 64 (words - 1) gets status -2: schedule not recorded in full). */
void orc_follow(const orc_mech *m, long n, const double *rho, const double *e0, double *T,
                double *Y, double dt, const orc_opts *o, const unsigned long long *trace,
                int words, int *status, int *level, int *iters, unsigned long long *sched,
                int nthreads);

/* Schedule hash: h0 = ORC_SCHED_SEED, then h = (h ^ (2 l + accepted)) * ORC_SCHED_PRIME per
 * sub-step attempt at level l (FNV-1a over the attempt codes). */
#define ORC_SCHED_SEED 0xcbf29ce484222325ULL
#define ORC_SCHED_PRIME 0x100000001b3ULL

/* e0[n] = e(Y, T) per cell. */
void orc_energy_batch(const orc_mech *m, long n, const double *T, const double *Y, double *e0);

/* Backward-Euler residual G = x - x_prev - h f(x), evaluated in long double; returns
 * max_i |G_i| / (atol_i + rtol |x_i|) and writes G (as double) if G_out != NULL. */
double orc_residual_ld(const orc_mech *m, double rho, const double *x_prev, const double *x,
                       double h, const orc_opts *o, double *G_out);

/* Term scale of the species rows of G at state x (for the parity floor):
 * S_s = |Y_prev,s| + h (M_s/rho_cgs) sum_r |nu_rs| |Mconc_r| (|qf_r| + |qb_r|). */
void orc_term_scale(const orc_mech *m, double rho, const double *Y_prev, const double *x,
                    double h, double *S);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
