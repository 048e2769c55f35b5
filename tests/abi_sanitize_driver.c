/*
 * abi_sanitize_driver.c -- drives the host runtime of libkzk (api.cpp, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer on the host side)
 * through the paths that need no GPU: status strings, null plans and
 * arguments, every parameter rejection (single solves and plans), and plan
 * creation on a machine without a usable device, which fails in its first
 * device call and must release what it built.  Exit status 0 when every
 * call returns the documented error class; a sanitizer finding aborts.
 */
#include <stdio.h>
#include <string.h>

#include "../include/kzk.h"

static int bad = 0;

static void expect(int cond, const char *what) {
    if (!cond) {
        fprintf(stderr, "unexpected result: %s\n", what);
        bad = 1;
    }
}

static kzk_params base(void) {
    kzk_params p;
    memset(&p, 0, sizeof(p));
    p.n_tau = 64; p.n_y = 32;
    p.tau0 = -4.0; p.L_tau = 8.0; p.y0 = -8.0; p.L_y = 16.0;
    p.x0 = 0.0; p.h = 1e-3; p.dtype = KZK_F32;
    p.D = 0.05; p.A = 0.0; p.nl = 1.0; p.weno_eps = 1e-6; p.cfl_max = 1.0;
    return p;
}

int main(void) {
    for (int s = -1; s <= 9; ++s) expect(kzk_status_str((kzk_status)s) != NULL, "status string");

    kzk_plan *plan = NULL;
    kzk_params p = base();
    expect(kzk_create(NULL, 1, NULL, &plan) == KZK_ERR_ARG, "null params");
    expect(kzk_create(&p, 0, NULL, &plan) == KZK_ERR_ARG, "no solves");
    expect(kzk_create(&p, 1, NULL, NULL) == KZK_ERR_ARG, "null out");
    expect(kzk_step(NULL, NULL, 0, 1) == KZK_ERR_ARG, "step on null plan");
    expect(kzk_adjoint(NULL, NULL, NULL, 0, 1, 1, NULL) == KZK_ERR_ARG, "adjoint on null plan");
    expect(kzk_poll(NULL) == KZK_ERR_ARG, "poll on null plan");
    expect(kzk_inst_offset(NULL, 0) == (size_t)-1, "offset on null plan");
    expect(kzk_set_y_threads(NULL, 256) == KZK_ERR_ARG, "y threads on null plan");
    expect(kzk_set_tau_threads(NULL, 256) == KZK_ERR_ARG, "tau threads on null plan");
    expect(kzk_autotune(NULL, NULL, 1) < 0, "autotune on null plan");
    expect(kzk_profile_enable(NULL, 1) == KZK_ERR_ARG, "profile on null plan");
    expect(kzk_eval_b(NULL, NULL, 0, NULL) == KZK_ERR_ARG, "eval_b on null plan");
    kzk_destroy(NULL);

    /* rejections before any device work */
    const int bad_tau[] = {16, 48, 96, 112, 480, 16384, 14336};
    for (unsigned i = 0; i < sizeof(bad_tau) / sizeof(bad_tau[0]); ++i) {
        kzk_params q = base();
        q.n_tau = bad_tau[i];
        expect(kzk_create(&q, 1, NULL, &plan) == KZK_ERR_SIZE && !plan, "n_tau rejected");
    }
    {
        kzk_params q = base();
        q.n_y = 448;
        expect(kzk_create(&q, 1, NULL, &plan) == KZK_ERR_SIZE, "n_y rejected");
        q = base(); q.h = 0.0;
        expect(kzk_create(&q, 1, NULL, &plan) == KZK_ERR_ARG, "h rejected");
        q = base(); q.vel = 1;
        expect(kzk_create(&q, 1, NULL, &plan) == KZK_ERR_ARG, "vel without a field rejected");
        q = base(); q.state_fp64 = 1; q.reg_eps = 1e-7;
        expect(kzk_create(&q, 1, NULL, &plan) == KZK_ERR_ARG, "state_fp64 with reg_eps rejected");
        kzk_params two[2] = {base(), base()};
        two[0].n_tau = 448; two[1].n_tau = 896;
        expect(kzk_create(two, 2, NULL, &plan) == KZK_ERR_SIZE, "two 7 2^k lengths rejected");
        two[1] = base(); two[1].dtype = KZK_F64; two[0] = base();
        expect(kzk_create(two, 2, NULL, &plan) == KZK_ERR_ARG, "mixed dtypes rejected");
        expect(kzk_step_noalloc(&q, 1, NULL, NULL, 0, 1) != KZK_OK, "noalloc with a bad argument");
    }

    /* valid plans: without a device the first device call fails; the
       partial plan is released (the sanitizer checks the unwinding) */
    {
        double D[4] = {0.05, 0.05, 0.05, 0.05}, nl[5] = {1, 1, 1, 1, 1}, phi[3] = {0.1, 0.2, 0.3},
               th[3] = {1.0, 2.0, 3.0};
        kzk_params q[3] = {base(), base(), base()};
        q[1].n_tau = 256; q[1].n_y = 128; q[1].D_step = D; q[1].nl_node = nl; q[1].n_steps_max = 4;
        q[2].n_tau = 32; q[2].n_y = 16; q[2].scheme = 0;
        kzk_status st = kzk_create(q, 3, NULL, &plan);
        if (st == KZK_OK) kzk_destroy(plan);   /* a machine with a device */
        plan = NULL;
        kzk_params g = base();
        g.n_tau = 448; g.vel = 1; g.vel_modes = 3; g.vel_phi = phi; g.vel_theta = th;
        g.vel_lambda = 6.86; g.vel_sigma_u = 3.0; g.vel_c0 = 343.0; g.n_steps_max = 4;
        g.D_step = D; g.nl_node = nl;
        st = kzk_create(&g, 1, NULL, &plan);
        if (st == KZK_OK) kzk_destroy(plan);
    }
    if (!bad) printf("host runtime sanitize driver: every call returned as documented\n");
    return bad;
}
