/*
 * sanitize_driver.c -- exercises every entry point of the oracle on small
 * inputs so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (gcc -fsanitize=address,undefined) can check its memory accesses and
 * arithmetic: transforms of power-of-two and mixed lengths, the phi-functions
 * and the symbol (plain and regularised), WENO5 b and its adjoint, the
 * velocity field and b with transport, marches of both schemes with the
 * per-line and the global LF speed and with a prescribed right-hand side,
 * and the checkpointed adjoint.  TEST INFRASTRUCTURE ONLY, like the oracle.
 *
 * Exit status 0 when every result is finite; a sanitizer finding aborts.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "kzk_oracle.h"

static unsigned long long rng_state = 0x9e3779b97f4a7c15ull;

/* SplitMix64 (Steele, Lea, Flood 2014), uniform in [-1, 1) */
static double urand(void) {
    unsigned long long z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int bad = 0;

static void check(const char *what, const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            fprintf(stderr, "%s: non-finite value at %zu\n", what, i);
            bad = 1;
            return;
        }
}

static double *field(size_t n, double amp) {
    double *a = malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) a[i] = amp * urand();
    return a;
}

static orc_cfg cfg(int nt, int ny, int nsteps, double *D, double *nl) {
    orc_cfg c;
    memset(&c, 0, sizeof(c));
    c.nt = nt; c.ny = ny;
    c.tau0 = -4.0; c.Lt = 8.0; c.y0 = -8.0; c.Ly = 16.0;
    c.x0 = 0.5; c.h = 1e-3; c.A = 1e-4; c.eps = 1e-6;
    c.Dbar = D; c.nl = nl; c.nsteps_max = nsteps;
    for (int i = 0; i < nsteps; ++i) D[i] = 0.05 * (1.0 + 0.2 * urand());
    for (int i = 0; i <= nsteps; ++i) nl[i] = 1.0 + 0.2 * urand();
    return c;
}

int main(void) {
    /* transforms: lengths 1 .. 64 (every factorisation the oracle takes), 448, 7 2^5 */
    for (int n = 1; n <= 64; ++n) {
        double *x = field(2 * (size_t)n, 1.0);
        orc_fft(x, n, -1);
        orc_fft(x, n, 1);
        check("fft", x, 2 * (size_t)n);
        free(x);
    }
    {
        double *a = field(2 * 448 * 8, 1.0);
        orc_fft2(a, 8, 448, -1);
        orc_fft2(a, 8, 448, 1);
        check("fft2", a, 2 * 448 * 8);
        free(a);
    }
    /* phi-functions across the series / closed-form switch */
    for (int i = 0; i < 200; ++i) {
        double zr = 3.0 * urand(), zi = 3.0 * urand(), r, im;
        for (int k = 0; k < 3; ++k) {
            orc_phi(k, zr, zi, &r, &im);
            double v[2] = {r, im};
            check("phi", v, 2);
        }
    }
    enum { NS = 6 };
    double D[NS], nl[NS + 1];
    for (int pass = 0; pass < 2; ++pass) {
        const int nt = pass ? 224 : 64, ny = pass ? 14 : 16;
        orc_cfg c = cfg(nt, ny, NS, D, nl);
        const size_t N = (size_t)nt * ny;
        /* symbol, plain and regularised, every mode */
        for (int reg = 0; reg < 2; ++reg) {
            c.reg_eps = reg ? 1e-8 : 0.0;
            for (int m = 0; m <= nt / 2; ++m)
                for (int n = 0; n < ny; ++n) {
                    double v[2];
                    orc_symbol(&c, m, n, 0.05, &v[0], &v[1]);
                    check("symbol", v, 2);
                }
        }
        c.reg_eps = 0.0;
        /* WENO5 b and its adjoint on one line */
        double *u = field(N, 1.0), *b = malloc(N * sizeof(double)), *g = field(nt, 1.0);
        double *ub = malloc(nt * sizeof(double)), ab = 0.0;
        orc_weno_b(u, nt, c.Lt / nt, 1.0, 1.0, c.eps, b);
        orc_weno_b_adj(u, nt, c.Lt / nt, 1.0, 1.0, c.eps, g, ub, &ab);
        check("weno_b", b, nt);
        check("weno_b_adj", ub, nt);
        /* velocity field and b with transport: the random field and profiles */
        double phi[40], theta[40], prof[3 * 16];
        for (int i = 0; i < 40; ++i) { phi[i] = 3.0 * (urand() + 1.0); theta[i] = 3.0 * (urand() + 1.0); }
        for (int i = 0; i < 3 * ny; ++i) prof[i] = 0.01 * urand();
        c.vel_modes = 40; c.vel_phi = phi; c.vel_theta = theta;
        c.vel_lambda = 6.86; c.vel_sigma_u = 3.0; c.vel_c0 = 343.0; c.vel_prof = prof;
        for (int vel = 0; vel < 3; ++vel) {
            c.vel = vel;
            if (vel) {
                double o[3];
                orc_velocity(&c, 0.7, 1.3, o);
                check("velocity", o, 3);
            }
            orc_eval_b(&c, 0.7, 0.9, u, b);
            check("eval_b", b, N);
        }
        /* marches: both schemes, plain and regularised, per-line and global LF speed, transport */
        for (int variant = 0; variant < 6; ++variant) {
            c.scheme = variant == 1 || variant == 4;
            c.reg_eps = variant >= 3 ? 1e-8 : 0.0;
            c.lf_global = variant == 2;
            c.vel = variant == 5 ? 1 : 0;
            double *w = malloc(N * sizeof(double));
            for (size_t i = 0; i < N; ++i) w[i] = 0.5 * u[i];
            if (orc_run(&c, w, 0, NS) != 0) { fprintf(stderr, "run variant %d failed\n", variant); bad = 1; }
            check("run", w, N);
            free(w);
        }
        c.scheme = 0; c.reg_eps = 0.0; c.lf_global = 0; c.vel = 0;
        /* prescribed right-hand side */
        {
            double *f0 = field(N, 0.1), *f1 = field(N, 0.1), *w = field(N, 0.5);
            c.force0 = f0; c.force1 = f1;
            if (orc_run(&c, w, 1, NS - 1) != 0) { fprintf(stderr, "forced run failed\n"); bad = 1; }
            check("forced run", w, N);
            c.force0 = c.force1 = NULL;
            free(f0); free(f1); free(w);
        }
        /* adjoint with checkpoints every 2 steps */
        {
            double *u0 = field(N, 0.5), *lam = field(N, 1.0);
            if (orc_adjoint(&c, u0, lam, 0, NS, 2) != 0) { fprintf(stderr, "adjoint failed\n"); bad = 1; }
            check("adjoint", lam, N);
            free(u0); free(lam);
        }
        free(u); free(b); free(g); free(ub);
    }
    if (!bad) printf("oracle sanitize driver: all results finite\n");
    return bad;
}
