/*
 * kzk_oracle.h -- plain FP64 CPU oracle for the exponential-integrator/WENO5
 * time step of the KZK-type sonic-boom equation (Einkemmer, Ostermann,
 * Residori, arXiv 2103.06080).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code; only the test-suite, the smoke check and the CPU baseline leg
 * of the benchmark use it.  It shares no code, header or table with the HIP
 * path.
 *
 * Equation (build notation; the paper's (sigma, rho, theta, V) are (x, y, tau, u)):
 *
 *     u_x = L u + b(x, u),
 *     L   = (D/2) d_tau^{-1} d_yy + A d_tau^2              (Sec. 3.3, eq. (15)/(17))
 *     b   = -nl(x) d_tau (u^2 / 2)                          (Sec. 3.3, eq. (16), Burgers part)
 *
 * on the periodic box [tau0, tau0+Lt) x [y0, y0+Ly) (Sec. 3.4), stepped with
 * the two-stage exponential Runge-Kutta method ExpRK22 (Sec. 3.3, eq. (19)) in
 * Fourier space (Sec. 3.4, eq. (20), Algorithm 2); b is discretised with WENO5
 * (Sec. 3.4, Jiang-Shu weights, Lax-Friedrichs flux splitting).
 *
 * Arrays are row-major [ny][nt]: element (j, k) = u(tau_k, y_j), tau contiguous.
 */
#ifndef KZK_ORACLE_H
#define KZK_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int    nt, ny;          /* grid points along tau and y (even; powers of two, or
                               2^a times an odd factor such as the paper's 7 2^k)     */
    double tau0, Lt;        /* tau box [tau0, tau0 + Lt)                             */
    double y0, Ly;          /* y box   [y0, y0 + Ly)                                 */
    double x0, h;           /* marching origin and step                              */
    double A;               /* absorption coefficient, A >= 0                        */
    double eps;             /* WENO epsilon (1e-6)                                   */
    int    lf_global;       /* 0: LF alpha per tau-line, 1: one alpha for the field  */
    const double *Dbar;     /* [nsteps_max]   diffraction coefficient of step n       */
    const double *nl;       /* [nsteps_max+1] Burgers coefficient at node x_n         */
    int    nsteps_max;
    /* Optional prescribed right-hand side used instead of WENO Burgers:
       b(x, u) = force0 + x * force1 (both [ny][nt]); NULL for the normal method. */
    const double *force0, *force1;
    int    scheme;          /* 0: ExpRK22 (Sec. 3.3 eq. (19)); 1: exponential Euler (Sec. 3.3)  */
    double reg_eps;         /* 0: mean tau-mode zeroed (l = 0 there, F(b)(0, .) := 0);
                               > 0: regularised multiplier of Sec. 3.4, 1/(i kt) replaced by
                               1/(i kt + reg_eps/(4 pi)) at every tau-mode, F(b) kept whole    */
    /* Transport by the velocity field U = (U_par, U_perp)(x, y) of Sec. 2 (b of Sec. 3.3 eq. (16),
       conservative form of Sec. 3.4 eq. (21)-(22)):
         b = -d_tau(nl u^2/2 - 2 pi U_par u) - d_y(U_perp u) + (d_y U_perp) u.
       vel = 0: no transport (b is the Burgers term only);
       vel = 1: the random field of Algorithm 1 with vel_modes modes, phases vel_phi[n] and
                angles vel_theta[n] (uniform in [0, 2 pi)), r = vel_lambda (x, y), length scale
                L = 4 vel_lambda, K_n equispaced in [0.1/L, 9/L], |U~(K_n)| = sqrt(E(K_n)/N),
                E(K) = sigma_u^2 K^3 L^4 exp(-(K L/2)^2) / 8, normalised by vel_c0;
       vel = 2: x-independent profiles vel_prof[0..2][ny] = U_par, U_perp, d_y U_perp at y_j. */
    int    vel;
    int    vel_modes;
    const double *vel_phi, *vel_theta;
    double vel_lambda, vel_sigma_u, vel_c0;
    const double *vel_prof;
} orc_cfg;

/* In-place complex FFT of length n with unit stride: radix-2 for powers of
   two, radix-2 steps down to the odd factor (taken by its direct sum) else.
   sign = -1: X_k = sum_j x_j e^{-2 pi i jk/n}; sign = +1: the conjugate kernel.
   No normalisation in either direction. */
void orc_fft(double *x_interleaved, int n, int sign);

/* Unnormalised 2D FFT of a complex [ny][nt] array (rows along tau, then columns). */
void orc_fft2(double *a_interleaved, int ny, int nt, int sign);

/* phi_k(z) for k = 0, 1, 2 (phi_0 = e^z), Sec. 3.3 eq. (19) and Sec. 3.4 eq. (20). */
void orc_phi(int k, double zr, double zi, double *out_r, double *out_i);

/* Linear symbol l(m, n) of L at tau-index m, y-index n (Sec. 3.4, z_jk/h):
   l = i * Dbar * ky^2 / (2 kt) - A kt^2, with l = 0 at m = 0 and the
   diffraction part dropped at the tau-Nyquist m = nt/2; with reg_eps > 0,
   l = -(Dbar/2) ky^2 / (i kt + reg_eps/(4 pi)) - A kt^2 at every m but the
   tau-Nyquist. */
void orc_symbol(const orc_cfg *c, int m, int n, double Dbar, double *lr, double *li);

/* WENO5-JS / Lax-Friedrichs discretisation of b = -nl d_tau(u^2/2) on one
   periodic tau-line of n points, with the splitting speed alpha given. */
void orc_weno_b(const double *u, int n, double dtau, double nl, double alpha,
                double eps, double *b);

/* Transpose of the Jacobian of orc_weno_b at u (alpha frozen), applied to g,
   plus the adjoint of alpha, returned in *alpha_bar (so that the full
   directional derivative is db = J du + (db/dalpha) dalpha). */
void orc_weno_b_adj(const double *u, int n, double dtau, double nl, double alpha,
                    double eps, const double *g, double *u_bar, double *alpha_bar);

/* Velocity field at (x, y): out = (U_par, U_perp, d_y U_perp) (cfg.vel = 1 or 2). */
void orc_velocity(const orc_cfg *c, double x, double y, double out[3]);

/* b(x, u) on the whole field [ny][nt] with the Burgers coefficient nl (the
   same b the stepper uses: WENO5/LF Burgers term, plus the transport terms when
   cfg.vel != 0). */
void orc_eval_b(const orc_cfg *c, double x, double nl, const double *u, double *b);

/* Advance the physical field u [ny][nt] by n_steps ExpRK22 steps starting at
   step index first (x_n = x0 + n h).  Returns 0 on success. */
int orc_run(const orc_cfg *c, double *u, int first, int n_steps);

/* Wall time in seconds of the step loop of the most recent orc_run call
   (the initial and final transforms excluded). */
double orc_last_step_seconds(void);

/* Discrete adjoint of orc_run: given u0 (the field at step `first`) and
   lam = dL/du at step first + n_steps, overwrite lam with dL/du0.
   Checkpoints every ckpt steps, recomputing each segment forward.
   ExpRK22 with the mean mode zeroed only (returns -3 otherwise). */
int orc_adjoint(const orc_cfg *c, const double *u0, double *lam, int first,
                int n_steps, int ckpt);

#ifdef __cplusplus
}
#endif
#endif
