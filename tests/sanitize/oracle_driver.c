/* Drives the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host only): small
 * solves of both vehicles with every belief reading, the repair, the update with non-finite
 * costs, the distance, moments and the local repair.  Exit status 0 when every call returns. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/bss_oracle.h"

static void base(orc_params* p)
{
    memset(p, 0, sizeof(*p));
    p->m = 1500; p->Iz = 2500; p->lf = 1.2; p->lr = 1.6; p->Cf = 5e4; p->Cr = 5e4; p->mu = 1.0;
    p->g = 9.81; p->v_min = 3.0; p->dt = 0.05; p->steer_max = 0.4; p->accel_max = 4.0;
    p->sigma_eps[0] = 0.1; p->sigma_eps[1] = 1.0;
    p->sigma_w[0] = 0.1; p->sigma_w[1] = 0.1; p->sigma_w[2] = 0.05;
    p->K = 7; p->M = 13; p->T = 6; p->delta = 0.05; p->gamma = 0.2; p->lambda = 1.0;
    p->gamma_u = 1.0; p->v_goal = 6.0; p->q_vx = 1.0; p->q_ey = 0.1; p->q_epsi = 1.0;
    p->C_cbf = 100.0; p->C_obs = 1000.0; p->phi_scale = 1.0; p->ell_a = 30; p->ell_b = 20;
    p->half_width = 2.0; p->shield_gmin = 0.05; p->shield_fd = 1e-2; p->seed = 7;
}

int main(void)
{
    orc_params p;
    base(&p);
    double x0[6] = {30.0, 0.0, 1.5707963267948966, 5.0, 0.0, 0.0};
    double Sigma0[36] = {0};
    for (int i = 0; i < 6; ++i) Sigma0[i * 6 + i] = 1e-3;
    int T = p.T, K = p.K;
    double* v = calloc((size_t)T * 2, sizeof(double));
    double* u = malloc(sizeof(double) * (size_t)K * T * 2);
    double* mom = malloc(sizeof(double) * (size_t)K * (T + 1) * ORC_NMOM);
    double* S = malloc(sizeof(double) * (size_t)K);
    double stats[4];
    for (int variant = 0; variant < 6; ++variant) {
        base(&p);
        if (variant == 1) p.belief = 1;
        if (variant == 2) { p.belief = 2; p.M = 12; }
        if (variant == 3) { p.shield_iters = 2; p.n_obs = 1; p.obs[0] = 30.3; p.obs[1] = 1.0; p.obs[2] = 0.3; }
        if (variant == 4) { p.n_con = 2; p.con_a[3] = 1.0; p.con_b[0] = 6.0; p.con_a[11] = 1.0; p.con_b[1] = 0.5; p.shield_iters = 1; }
        if (variant == 5) { p.local_repair = 1; p.shield_iters = 2; p.crn = 1; p.sigma_w_speed = 0.1; }
        memset(v, 0, sizeof(double) * (size_t)T * 2);
        if (orc_solve(&p, 3, x0, variant == 1 ? Sigma0 : NULL, v, u, mom, S, stats, 3) != 0) return 2;
        for (int i = 0; i < T * 2; ++i) if (!isfinite(v[i])) return 3;
    }
    /* every cost non-finite: the update reports it and keeps v */
    base(&p);
    for (int k = 0; k < K; ++k) S[k] = NAN;
    if (orc_update(&p, S, u, v, stats) != 1) return 4;
    /* distance on the axes, the centre and far away */
    double sd, n[2];
    double pts[5][2] = {{0, 0}, {31, 0}, {0, -21}, {1e6, 3}, {-29.5, 1e-300}};
    for (int i = 0; i < 5; ++i) orc_ellipse_sdf(30, 20, pts[i][0], pts[i][1], &sd, n);
    /* the 8-state vehicle */
    base(&p);
    p.vehicle = 1; p.m = 22; p.Iz = 1.1; p.lf = 0.34; p.lr = 0.23; p.mu = 0.9; p.v_min = 2.0;
    p.Rw = 0.095; p.Iw = 0.3; p.T_max = 8; p.pac_B = 10; p.pac_C = 1.9; p.pac_D = 1; p.pac_E = 0.97;
    p.track_len = 120; p.kappa_amp = 0.8; p.n_sub = 4; p.accel_max = 1.0;
    double y0[8] = {5, 0, 0, 5 / 0.095, 5 / 0.095, 0, 0, 10};
    double* rec = malloc(sizeof(double) * (size_t)K * (T + 1) * ORC8_NREC);
    memset(v, 0, sizeof(double) * (size_t)T * 2);
    if (orc8_solve(&p, 1, y0, v, u, rec, S, stats, 2) != 0) return 5;
    p.shield_iters = 2;
    double uu[2] = {0.1, 0.5};
    orc8_repair(&p, 1.64, rec, uu);
    free(rec);
    free(v);
    free(u);
    free(mom);
    free(S);
    puts("oracle driver: ok");
    return 0;
}
