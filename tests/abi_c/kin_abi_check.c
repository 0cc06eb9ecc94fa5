/* kin_abi_check.c -- drives libkin through its C ABI alone (no Python, no torch): a two-species
 * isomerisation A <=> B whose backward-Euler step has a closed form,
 *   Y_A = Y_eq + (Y_A,n - Y_eq) / (1 + (k_f + k_b) dt),  Y_eq = k_b / (k_f + k_b),  k_b = k_f / K,
 * with identical NASA-7 sets except a7, so K is the same at every temperature and T does not
 * move (Sec. 3.2: forward rate, equilibrium constant, implicit step).  Exit status 0 on
 * success.  Test infrastructure: built by the build entry point, run by a GPU test. */
#include <math.h>
#include <stdio.h>

#include "kin.h"

#define CHECK(call)                                                                      \
    do {                                                                                 \
        kin_status s_ = (call);                                                          \
        if (s_ != KIN_OK) {                                                              \
            fprintf(stderr, "%s failed: status %d: %s\n", #call, (int)s_, kin_last_error()); \
            return 2;                                                                    \
        }                                                                                \
    } while (0)

int main(void)
{
    const double kf = 1e9, K = 0.3, dt = 1e-6, T0 = 298.15;
    const double cp = 3.5, hf = -1000.0, s0 = 30.0;
    double M[2] = {2.016, 2.016};
    int8_t elem[2] = {2, 2};
    double nasa[2 * 2 * 7];
    for (int s = 0; s < 2; ++s)
        for (int r = 0; r < 2; ++r) {
            double *a = nasa + (s * 2 + r) * 7;
            a[0] = cp;
            a[1] = a[2] = a[3] = a[4] = 0.0;
            a[5] = hf - cp * T0;
            a[6] = s0 - cp * log(T0) + (s == 1 ? log(K) : 0.0);
        }
    double T_mid[2] = {1000.0, 1000.0};
    int32_t reac_idx[3] = {0, -1, -1}, reac_nu[3] = {1, 0, 0};
    int32_t prod_idx[3] = {1, -1, -1}, prod_nu[3] = {1, 0, 0};
    double A[1] = {kf}, b[1] = {0.0}, Ta[1] = {0.0};
    int32_t rev[1] = {1}, tb[1] = {-1};
    kin_mech_desc d = {2, 1, 1, 0, M, elem, nasa, T_mid, reac_idx, reac_nu, prod_idx, prod_nu,
                       A, b, Ta, rev, tb, NULL};

    kin_ctx *ctx = NULL;
    kin_ctx_opts o = {0, 0, NULL, 0};
    CHECK(kin_create(&ctx, &o));
    int32_t mid = -1, iid = -1;
    CHECK(kin_mech_upload(ctx, &d, &mid));

    enum { n = 3 };
    double rho[n] = {0.3, 0.05, 1.0}, T[n] = {1500.0, 900.0, 2500.0};
    double Y[2 * n] = {0.9, 0.2, 0.5, 0.1, 0.8, 0.5};
    CHECK(kin_state_upload(ctx, mid, n, rho, T, Y, NULL, KIN_MEM_HOST, NULL, &iid));
    CHECK(kin_advance(ctx, &iid, &dt, 1, KIN_FP64, NULL, NULL));
    double To[n], Yo[2 * n];
    int32_t st[n], lv[n], it[n];
    CHECK(kin_download(ctx, iid, To, Yo, NULL, st, lv, it, KIN_MEM_HOST, NULL));

    const double kb = kf / K, yeq = kb / (kf + kb);
    int bad = 0;
    for (int c = 0; c < n; ++c) {
        const double yA = yeq + (Y[c] - yeq) / (1.0 + (kf + kb) * dt);
        const double err = fabs(Yo[c] - yA) / yA, errT = fabs(To[c] - T[c]) / T[c];
        printf("cell %d: status %d iters %d  Y_A %.17g (closed form %.17g, rel err %.2e)  T rel err %.2e\n",
               c, st[c], it[c], Yo[c], yA, err, errT);
        if (st[c] != KIN_CELL_OK || !(err <= 1e-13) || !(errT <= 1e-13)) bad = 1;
    }
    CHECK(kin_instance_release(ctx, iid));
    CHECK(kin_mech_release(ctx, mid));
    kin_destroy(ctx);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
