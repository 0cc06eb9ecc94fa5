/*
 * kin_oracle.c -- plain FP64 CPU oracle of the per-cell implicit chemical-kinetics update
 * (Le & Cambier, arXiv:1110.4903, Sec. 3.2 and Sec. 4.2).  TEST INFRASTRUCTURE ONLY: see
 * kin_oracle.h.  Written for clarity, not speed: dense loops, no blocking or fusion, built
 * with -O2 -ffp-contract=off, OpenMP only over independent cells.
 *
 * Readings of points the paper leaves open (each is also listed with the design notes):
 *  - unknowns x = (Y_1..Y_Ns, T) of a constant-density, constant-internal-energy cell; the
 *    implicit system (I - h df/dx) dx = -G is iterated as Newton's method on backward Euler,
 *    G = x - x_prev - h f(x), starting from x_prev (the paper's point-implicit step is the
 *    first Newton iteration);
 *  - convergence when |dx_i| <= atol_i + rtol |x_i| for every i after the update (each
 *    Newton iteration is counted when it starts);
 *  - failure of a sub-step: no convergence within k_max iterations, a non-finite value, an
 *    exactly zero pivot, T outside [200, 6000] K, a converged iterate with a mass fraction
 *    below -y_neg, or no root of e(Y, T) = e0 in [200, 6000] K;
 *  - sub-stepping is dyadic: sub-step h = dt 2^-l starts at l = 0; a failed sub-step is
 *    retried from the last accepted state at l + 1; after an accepted sub-step l drops by
 *    one when the elapsed time is a multiple of the doubled step; l > L_max fails the cell,
 *    which keeps its input state, and so does a cell that has used max_iters Newton
 *    iterations before the end of its step;
 *  - after each accepted sub-step T is reset to the root of e(Y, T) = e0;
 *  - R is the universal gas constant and P_a one standard atmosphere.
 */
#include "kin_oracle.h"

#include <math.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_RU 8.31446261815324          /* J/(mol K) */
#define ORC_RU_CGS 8.31446261815324e7    /* erg/(mol K) */
#define ORC_PATM_CGS 1.01325e6           /* dyn/cm^2 */
#define ORC_T_MIN 200.0
#define ORC_T_MAX 6000.0

/* ---- double instantiation ---- */
#define REAL double
#define FN(name) name##_d
#define EXP exp
#define LOG log
#define POW pow
#include "kin_oracle_eval.inc"
#undef REAL
#undef FN
#undef EXP
#undef LOG
#undef POW

/* ---- long double instantiation (residual check only) ---- */
#define REAL long double
#define FN(name) name##_ld
#define EXP expl
#define LOG logl
#define POW powl
#include "kin_oracle_eval.inc"
#undef REAL
#undef FN
#undef EXP
#undef LOG
#undef POW

void orc_default_opts(orc_opts *o)
{
    o->rtol = 1e-12;
    o->atol_Y = 1e-20;
    o->atol_T = 1e-9;
    o->y_neg = 1e-10;
    o->k_max = 10;
    o->L_max = 40;
    o->max_iters = 100000;
    o->diverge_ratio = 2.0;
    o->point_implicit = 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_species_thermo(const orc_mech *m, double T, double *cp_R, double *h_RT, double *s_R,
                        double *dcpR_dT)
{
    thermo_d(m, T, cp_R, h_RT, s_R, dcpR_dT);
}

double orc_mix_energy(const orc_mech *m, const double *Y, double T)
{
    double h_RT[ORC_NS_MAX];
    thermo_d(m, T, 0, h_RT, 0, 0);
    double e = 0;
    for (int s = 0; s < m->ns; ++s)
        e += Y[s] * ORC_RU * T * (h_RT[s] - 1.0) / (m->M[s] * 1e-3);
    return e;
}

double orc_mix_cv(const orc_mech *m, const double *Y, double T)
{
    double cp_R[ORC_NS_MAX];
    thermo_d(m, T, cp_R, 0, 0, 0);
    double cv = 0;
    for (int s = 0; s < m->ns; ++s)
        cv += Y[s] * ORC_RU * (cp_R[s] - 1.0) / (m->M[s] * 1e-3);
    return cv;
}

void orc_rates(const orc_mech *m, double rho, const double *Y, double T, double *kf, double *kb,
               double *Mconc, double *qf, double *qb, double *q, double *wdot)
{
    rates_d(m, rho, Y, T, kf, kb, Mconc, qf, qb, q, wdot, 0);
}

void orc_rhs(const orc_mech *m, double rho, const double *x, double *f)
{
    rhs_d(m, rho, x, f);
}

/* Net stoichiometric coefficient nu_rs = nu''_rs - nu'_rs of species s in reaction r. */
static int net_nu(const orc_mech *m, int r, int s)
{
    int v = 0;
    for (int j = 0; j < 3; ++j) {
        if (m->prod_idx[3 * r + j] == s) v += m->prod_nu[3 * r + j];
        if (m->reac_idx[3 * r + j] == s) v -= m->reac_nu[3 * r + j];
    }
    return v;
}

/* d/dc of k * prod_j c_{idx_j}^{nu_j}, accumulated into grad[ns] (product rule). */
static void mass_action_grad(const int *idx, const int *nu, double k, const double *c, double *grad)
{
    for (int j = 0; j < 3; ++j) {
        if (idx[j] < 0) continue;
        double term = k * nu[j] * ipow_d(c[idx[j]], nu[j] - 1);
        for (int i = 0; i < 3; ++i)
            if (i != j && idx[i] >= 0) term *= ipow_d(c[idx[i]], nu[i]);
        grad[idx[j]] += term;
    }
}

/* Analytic Jacobian of f = (dY/dt, dT/dt) with respect to x = (Y, T).
 *
 * Species rows: f_s = (M_s/rho_cgs) wdot_s and c_k = rho_cgs Y_k / M_k give
 *   df_s/dY_k = (M_s/M_k) sum_r nu_rs dQ_r/dc_k,   df_s/dT = (M_s/rho_cgs) sum_r nu_rs dQ_r/dT.
 * Rate derivatives: dQ_r/dc_k = [M]_r (dq_f/dc_k - dq_b/dc_k) + alpha_rk (q_f - q_b) for
 * third-body reactions; d ln k_f/dT = (beta + Ta/T)/T; d ln K_e/dT = (-sum nu + sum_s nu_rs
 * h_s/RT)/T (van 't Hoff), so dq_b/dT = q_b (d ln k_f/dT - d ln K_e/dT).
 * Energy row: f_T = -(sum_s e_s f_s)/c_v with de_s/dT = cv_s, dc_v/dY_k = cv_k,
 * dc_v/dT = sum_s Y_s dcv_s/dT. */
void orc_jacobian(const orc_mech *m, double rho, const double *x, double *J)
{
    int ns = m->ns, N = ns + 1;
    double T = x[ns];
    double rho_cgs = rho * 1e-3;
    double c[ORC_NS_MAX], cp_R[ORC_NS_MAX], h_RT[ORC_NS_MAX], s_R[ORC_NS_MAX], dcpR[ORC_NS_MAX];
    double wdot[ORC_NS_MAX], JT[ORC_NS_MAX], dqdc[ORC_NS_MAX], dpf[ORC_NS_MAX], dpb[ORC_NS_MAX];
    double *Jc = (double *)calloc((size_t)ns * ns, sizeof(double));
    for (int s = 0; s < ns; ++s) { c[s] = rho_cgs * x[s] / m->M[s]; wdot[s] = 0; JT[s] = 0; }
    thermo_d(m, T, cp_R, h_RT, s_R, dcpR);
    double Pa_RT = ORC_PATM_CGS / (ORC_RU_CGS * T);

    for (int r = 0; r < m->nr; ++r) {
        const int *ri = m->reac_idx + 3 * r, *rn = m->reac_nu + 3 * r;
        const int *pi = m->prod_idx + 3 * r, *pn = m->prod_nu + 3 * r;
        double kf = m->A[r] * pow(T, m->b[r]) * exp(-m->Ta[r] / T);
        double dlnkf = (m->b[r] + m->Ta[r] / T) / T;
        double kb = 0, dlnKc = 0;
        if (m->reversible[r]) {
            int dnu = 0;
            double dG_RT = 0, dH_RT = 0;
            for (int j = 0; j < 3; ++j) {
                if (pi[j] >= 0) { dnu += pn[j]; dG_RT += pn[j] * (h_RT[pi[j]] - s_R[pi[j]]); dH_RT += pn[j] * h_RT[pi[j]]; }
                if (ri[j] >= 0) { dnu -= rn[j]; dG_RT -= rn[j] * (h_RT[ri[j]] - s_R[ri[j]]); dH_RT -= rn[j] * h_RT[ri[j]]; }
            }
            double Kc = ipow_d(Pa_RT, dnu >= 0 ? dnu : 0) / ipow_d(Pa_RT, dnu < 0 ? -dnu : 0) * exp(-dG_RT);
            kb = kf / Kc;
            dlnKc = (-dnu + dH_RT) / T;
        }
        double pf = kf, pb = kb;
        for (int j = 0; j < 3; ++j) {
            if (ri[j] >= 0) pf *= ipow_d(c[ri[j]], rn[j]);
            if (pi[j] >= 0) pb *= ipow_d(c[pi[j]], pn[j]);
        }
        for (int k = 0; k < ns; ++k) { dpf[k] = 0; dpb[k] = 0; }
        mass_action_grad(ri, rn, kf, c, dpf);
        if (kb != 0) mass_action_grad(pi, pn, kb, c, dpb);
        double M = 1;
        const double *alpha = 0;
        if (m->tb[r] >= 0) {
            alpha = m->eff + (long)m->tb[r] * ns;
            M = 0;
            for (int s = 0; s < ns; ++s) M += alpha[s] * c[s];
        }
        double q = M * (pf - pb);
        for (int k = 0; k < ns; ++k) {
            dqdc[k] = M * (dpf[k] - dpb[k]);
            if (alpha) dqdc[k] += alpha[k] * (pf - pb);
        }
        double dqdT = M * (pf * dlnkf - pb * (dlnkf - dlnKc));
        for (int s = 0; s < ns; ++s) {
            int nu = net_nu(m, r, s);
            if (nu == 0) continue;
            wdot[s] += nu * q;
            JT[s] += nu * dqdT;
            for (int k = 0; k < ns; ++k) Jc[s * ns + k] += nu * dqdc[k];
        }
    }

    double fY[ORC_NS_MAX], es[ORC_NS_MAX], cvs[ORC_NS_MAX];
    double cv = 0, dcvdT = 0, de = 0;
    for (int s = 0; s < ns; ++s) {
        double Mkg = m->M[s] * 1e-3;
        fY[s] = m->M[s] * wdot[s] / rho_cgs;
        es[s] = ORC_RU * T * (h_RT[s] - 1.0) / Mkg;
        cvs[s] = ORC_RU * (cp_R[s] - 1.0) / Mkg;
        cv += x[s] * cvs[s];
        dcvdT += x[s] * ORC_RU * dcpR[s] / Mkg;
        de += es[s] * fY[s];
    }
    double fT = -de / cv;
    for (int s = 0; s < ns; ++s) {
        for (int k = 0; k < ns; ++k) J[s * N + k] = m->M[s] / m->M[k] * Jc[s * ns + k];
        J[s * N + ns] = m->M[s] * JT[s] / rho_cgs;
    }
    for (int k = 0; k < ns; ++k) {
        double acc = 0;
        for (int s = 0; s < ns; ++s) acc += es[s] * J[s * N + k];
        J[ns * N + k] = -(acc + fT * cvs[k]) / cv;
    }
    double acc = 0;
    for (int s = 0; s < ns; ++s) acc += cvs[s] * fY[s] + es[s] * J[s * N + ns];
    J[ns * N + ns] = -(acc + fT * dcvdT) / cv;
    free(Jc);
}

void orc_jacobian_fd(const orc_mech *m, double rho, const double *x, double *J)
{
    int ns = m->ns, N = ns + 1;
    double xp[ORC_NS_MAX + 1], fp[ORC_NS_MAX + 1], fm[ORC_NS_MAX + 1];
    double eps3 = cbrt(2.220446049250313e-16);
    for (int j = 0; j < N; ++j) {
        double scale = (j < ns) ? fmax(fabs(x[j]), 1e-2) : fabs(x[j]);
        double hj = eps3 * scale;
        memcpy(xp, x, sizeof(double) * N);
        xp[j] = x[j] + hj;
        volatile double hp = xp[j] - x[j];
        rhs_d(m, rho, xp, fp);
        xp[j] = x[j] - hj;
        volatile double hm = x[j] - xp[j];
        rhs_d(m, rho, xp, fm);
        for (int i = 0; i < N; ++i) J[i * N + j] = (fp[i] - fm[i]) / (hp + hm);
    }
}

int orc_lu_factor(int n, double *A, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double amax = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            if (fabs(A[i * n + k]) > amax) { amax = fabs(A[i * n + k]); p = i; }
        }
        piv[k] = p;
        if (amax == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
            }
        }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}

void orc_lu_solve(int n, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k) {
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    }
    for (int i = 1; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= LU[i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= LU[i * n + j] * b[j];
        b[i] = s / LU[i * n + i];
    }
}

int orc_invert_T(const orc_mech *m, const double *Y, double e0, double T_start, double *T_out)
{
    double T = T_start;
    for (int it = 0; it < 20; ++it) {
        double cv = orc_mix_cv(m, Y, T);
        if (!(cv > 0)) break;
        double dT = (orc_mix_energy(m, Y, T) - e0) / cv;
        T -= dT;
        if (!isfinite(T) || T < ORC_T_MIN || T > ORC_T_MAX) break;
        if (fabs(dT) <= 1e-13 * T) { *T_out = T; return 0; }
    }
    /* Bisection fallback: e is increasing in T where c_v > 0. */
    double lo = ORC_T_MIN, hi = ORC_T_MAX;
    double flo = orc_mix_energy(m, Y, lo) - e0, fhi = orc_mix_energy(m, Y, hi) - e0;
    if (!(flo <= 0 && fhi >= 0)) return -1;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * lo; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_mix_energy(m, Y, mid) - e0 > 0) hi = mid; else lo = mid;
    }
    *T_out = 0.5 * (lo + hi);
    return 0;
}

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
    return 1;
}

int orc_be_substep(const orc_mech *m, double rho, double e0, double *x, double h,
                   const orc_opts *o, int *iters, double *x_be)
{
    int ns = m->ns, N = ns + 1;
    double xk[ORC_NS_MAX + 1], f[ORC_NS_MAX + 1], d[ORC_NS_MAX + 1];
    int piv[ORC_NS_MAX + 1];
    double *A = (double *)malloc(sizeof(double) * N * N);
    int rc = -1;
    memcpy(xk, x, sizeof(double) * N);
    double r_prev = -1.0;  /* weighted norm of the previous update */
    for (int k = 0; k < o->k_max; ++k) {
        ++*iters;
        orc_rhs(m, rho, xk, f);
        orc_jacobian(m, rho, xk, A);
        if (!all_finite(f, N) || !all_finite(A, N * N)) break;
        for (int i = 0; i < N; ++i) {
            d[i] = -(xk[i] - x[i] - h * f[i]);
            for (int j = 0; j < N; ++j) A[i * N + j] = (i == j ? 1.0 : 0.0) - h * A[i * N + j];
        }
        if (!all_finite(d, N) || !all_finite(A, N * N)) break;
        if (orc_lu_factor(N, A, piv) != 0) break;
        orc_lu_solve(N, A, piv, d);
        for (int i = 0; i < N; ++i) xk[i] += d[i];
        if (!all_finite(xk, N)) break;
        if (xk[ns] < ORC_T_MIN || xk[ns] > ORC_T_MAX) break;
        int conv = 1;
        for (int i = 0; i < N; ++i) {
            double atol = (i < ns) ? o->atol_Y : o->atol_T;
            if (!(fabs(d[i]) <= atol + o->rtol * fabs(xk[i]))) conv = 0;
        }
        if (o->point_implicit) conv = 1;  /* the linearised step is taken as it is */
        if (!conv && o->diverge_ratio > 0) {
            double r = 0;
            for (int i = 0; i < N; ++i) {
                double atol = (i < ns) ? o->atol_Y : o->atol_T;
                double ri = fabs(d[i]) / (atol + o->rtol * fabs(xk[i]));
                if (ri > r) r = ri;
            }
            if (r_prev >= 0 && r > o->diverge_ratio * r_prev) break;  /* diverging */
            r_prev = r;
        }
        if (conv) {
            int neg = 0;
            if (!o->point_implicit)
                for (int s = 0; s < ns; ++s) if (xk[s] < -o->y_neg) neg = 1;
            if (neg) break;
            if (x_be) memcpy(x_be, xk, sizeof(double) * N);
            double T;
            if (orc_invert_T(m, xk, e0, xk[ns], &T) != 0) break;
            xk[ns] = T;
            memcpy(x, xk, sizeof(double) * N);
            rc = 0;
            break;
        }
    }
    free(A);
    return rc;
}

static unsigned long long sched_step(unsigned long long h, int l, int accepted)
{
    return (h ^ (unsigned long long)(2 * l + accepted)) * ORC_SCHED_PRIME;
}

int orc_advance_cell(const orc_mech *m, double rho, double e0, double *T, double *Y, long stride,
                     double dt, const orc_opts *o, int L_forced, int *level, int *iters,
                     unsigned long long *sched)
{
    int ns = m->ns, N = ns + 1;
    double xn[ORC_NS_MAX + 1], x[ORC_NS_MAX + 1];
    *level = 0;
    *iters = 0;
    *sched = ORC_SCHED_SEED;
    for (int s = 0; s < ns; ++s) xn[s] = Y[s * stride];
    xn[ns] = *T;
    if (!all_finite(xn, N) || !isfinite(rho) || !(rho > 0) || !isfinite(e0) || !isfinite(dt) ||
        !(dt >= 0) || xn[ns] < ORC_T_MIN || xn[ns] > ORC_T_MAX)
        return ORC_BAD_INPUT;
    memcpy(x, xn, sizeof(double) * N);
    int failed = 0;
    if (o->point_implicit) L_forced = 0;  /* one step over dt, no halving */
    if (L_forced >= 0) {
        /* Replay: exactly 2^L equal sub-steps, no adaptation. */
        double h = ldexp(dt, -L_forced);
        long nsub = 1L << L_forced;
        *level = L_forced;
        for (long j = 0; j < nsub; ++j) {
            if (*iters >= o->max_iters) return ORC_FAILED;
            int ok = orc_be_substep(m, rho, e0, x, h, o, iters, 0) == 0;
            *sched = sched_step(*sched, L_forced, ok);
            if (!ok) return ORC_FAILED;
        }
    } else {
        /* Time is counted in ticks of dt 2^-L_max, so every sub-step boundary is exact. */
        const long long end = 1LL << o->L_max;
        long long t = 0;
        int l = 0;
        while (t < end) {
            if (*iters >= o->max_iters) return ORC_FAILED;
            double h = ldexp(dt, -l);
            int ok = orc_be_substep(m, rho, e0, x, h, o, iters, 0) == 0;
            *sched = sched_step(*sched, l, ok);
            if (ok) {
                t += 1LL << (o->L_max - l);
                if (l > 0 && (t & ((1LL << (o->L_max - l + 1)) - 1)) == 0) --l;
            } else {
                failed = 1;
                ++l;
                if (l > *level) *level = l;
                if (l > o->L_max) { *level = o->L_max; return ORC_FAILED; }
            }
        }
    }
    for (int s = 0; s < ns; ++s) Y[s * stride] = x[s];
    *T = x[ns];
    return failed ? ORC_OK_HALVED : ORC_OK;
}

int orc_follow_cell(const orc_mech *m, double rho, double e0, double *T, double *Y, long stride,
                    double dt, const orc_opts *o, const unsigned long long *bits, long count,
                    int *level, int *iters, unsigned long long *sched)
{
    int ns = m->ns, N = ns + 1;
    double xn[ORC_NS_MAX + 1], x[ORC_NS_MAX + 1];
    *level = 0;
    *iters = 0;
    *sched = ORC_SCHED_SEED;
    for (int s = 0; s < ns; ++s) xn[s] = Y[s * stride];
    xn[ns] = *T;
    if (!all_finite(xn, N) || !isfinite(rho) || !(rho > 0) || !isfinite(e0) || !isfinite(dt) ||
        !(dt >= 0) || xn[ns] < ORC_T_MIN || xn[ns] > ORC_T_MAX)
        return ORC_BAD_INPUT;
    /* an accepted attempt is solved to convergence: no divergence test, at least 50 iterations */
    orc_opts solve = *o;
    solve.diverge_ratio = 0.0;
    if (solve.k_max < 50) solve.k_max = 50;
    memcpy(x, xn, sizeof(double) * N);
    const long long end = 1LL << o->L_max;
    long long t = 0;
    int l = 0, failed = 0;
    for (long j = 0; j < count && t < end; ++j) {
        int accepted = (int)((bits[j / 64] >> (j % 64)) & 1ULL);
        *sched = sched_step(*sched, l, accepted);
        if (accepted) {
            if (orc_be_substep(m, rho, e0, x, ldexp(dt, -l), &solve, iters, 0) != 0) return -1;
            t += 1LL << (o->L_max - l);
            if (l > 0 && (t & ((1LL << (o->L_max - l + 1)) - 1)) == 0) --l;
        } else {
            failed = 1;
            ++l;
            if (l > *level) *level = l;
            if (l > o->L_max) { *level = o->L_max; break; }
        }
    }
    if (t < end) return ORC_FAILED;
    for (int s = 0; s < ns; ++s) Y[s * stride] = x[s];
    *T = x[ns];
    return failed ? ORC_OK_HALVED : ORC_OK;
}

void orc_follow(const orc_mech *m, long n, const double *rho, const double *e0, double *T, double *Y,
                double dt, const orc_opts *o, const unsigned long long *trace, int words, int *status,
                int *level, int *iters, unsigned long long *sched, int nthreads)
{
    if (nthreads <= 0) nthreads = orc_num_threads();
    long i;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (i = 0; i < n; ++i) {
        const unsigned long long *tr = trace + (size_t)i * words;
        const long count = (long)tr[0];
        int lv = 0, it = 0, st;
        unsigned long long sh = ORC_SCHED_SEED;
        if (count > 64L * (words - 1)) st = -2;
        else st = orc_follow_cell(m, rho[i], e0[i], &T[i], &Y[i], n, dt, o, tr + 1, count, &lv, &it, &sh);
        status[i] = st;
        level[i] = lv;
        iters[i] = it;
        sched[i] = sh;
    }
}

void orc_advance(const orc_mech *m, long n, const double *rho, const double *e0, double *T,
                 double *Y, double dt, const orc_opts *o, int L_forced, int *status, int *level,
                 int *iters, unsigned long long *sched, int nthreads)
{
    if (nthreads <= 0) nthreads = orc_num_threads();
    long i;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (i = 0; i < n; ++i) {
        double e = e0 ? e0[i] : 0.0;
        if (!e0) {
            double y[ORC_NS_MAX];
            for (int s = 0; s < m->ns; ++s) y[s] = Y[s * n + i];
            e = orc_mix_energy(m, y, T[i]);
        }
        int lv, it;
        unsigned long long sh;
        int st = orc_advance_cell(m, rho[i], e, &T[i], &Y[i], n, dt, o, L_forced, &lv, &it, &sh);
        if (status) status[i] = st;
        if (level) level[i] = lv;
        if (iters) iters[i] = it;
        if (sched) sched[i] = sh;
    }
}

void orc_energy_batch(const orc_mech *m, long n, const double *T, const double *Y, double *e0)
{
    for (long i = 0; i < n; ++i) {
        double y[ORC_NS_MAX];
        for (int s = 0; s < m->ns; ++s) y[s] = Y[s * n + i];
        e0[i] = orc_mix_energy(m, y, T[i]);
    }
}

double orc_residual_ld(const orc_mech *m, double rho, const double *x_prev, const double *x,
                       double h, const orc_opts *o, double *G_out)
{
    int ns = m->ns, N = ns + 1;
    long double xl[ORC_NS_MAX + 1], f[ORC_NS_MAX + 1];
    for (int i = 0; i < N; ++i) xl[i] = x[i];
    rhs_ld(m, (long double)rho, xl, f);
    double worst = 0;
    for (int i = 0; i < N; ++i) {
        long double G = xl[i] - (long double)x_prev[i] - (long double)h * f[i];
        if (G_out) G_out[i] = (double)G;
        double atol = (i < ns) ? o->atol_Y : o->atol_T;
        double r = (double)(fabsl(G) / ((long double)atol + (long double)o->rtol * fabsl(xl[i])));
        if (r > worst) worst = r;
    }
    return worst;
}

void orc_term_scale(const orc_mech *m, double rho, const double *Y_prev, const double *x, double h,
                    double *S)
{
    int ns = m->ns;
    double *qf = (double *)malloc(sizeof(double) * m->nr * 3);
    double *qb = qf + m->nr, *Mc = qb + m->nr;
    double wdot[ORC_NS_MAX];
    rates_d(m, rho, x, x[ns], 0, 0, Mc, qf, qb, 0, wdot, 0);
    double rho_cgs = rho * 1e-3;
    for (int s = 0; s < ns; ++s) {
        double acc = 0;
        for (int r = 0; r < m->nr; ++r) {
            int nu = net_nu(m, r, s);
            if (nu) acc += fabs((double)nu) * fabs(Mc[r]) * (fabs(qf[r]) + fabs(qb[r]));
        }
        S[s] = fabs(Y_prev[s]) + h * m->M[s] / rho_cgs * acc;
    }
    free(qf);
}
