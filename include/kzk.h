/*
 * kzk.h -- C ABI of libkzk: the time step of the exponential-integrator /
 * WENO5 discretisation of the KZK-type sonic-boom equation (Einkemmer,
 * Ostermann, Residori, arXiv 2103.06080), hand-written HIP for MI355X (gfx950).
 *
 * Equation (the paper's sigma, rho, theta, V are x, y, tau, u here):
 *
 *     u_x = (D/2) d_tau^{-1} d_yy u + A d_tau^2 u - nl d_tau(u^2/2)
 *
 * i.e. the evolution form of Sec. 3.3 eq. (14) with the linear part L of
 * eq. (15)/(17) and the Burgers part of b (paper: D = 1/(2 pi), nl = -B).
 * The periodic (tau, y) box of Sec. 3.4 is marched in x with step h by
 * ExpRK22 in Fourier space (Sec. 3.3 eq. (19), Sec. 3.4 eq. (20),
 * Algorithm 2); b is discretised with WENO5 (Jiang-Shu weights, p = 2) and
 * Lax-Friedrichs flux splitting with speed alpha = |nl| max_tau |u| per line.
 *
 * Conventions shared by every entry point:
 *  - Fields are row-major [n_y][n_tau] (tau contiguous) device arrays of the
 *    plan's dtype (float or double): u[j * n_tau + k] = u(tau0 + k dtau, y0 + j dy).
 *  - The caller owns every device buffer it passes; the plan owns its
 *    workspace.  No call frees caller memory.
 *  - All work is enqueued on the plan's HIP stream; calls return without
 *    synchronising, except kzk_poll.
 *  - Errors are returned, never thrown; nothing aborts.  Argument errors are
 *    detected before anything is enqueued.  Conditions found on the device
 *    (CFL limit exceeded, non-finite values) are latched in a device status
 *    word and reported by kzk_poll.
 *  - Multiplier conventions: the mean tau-mode has l = 0 (E = 1, Phi1 = 1,
 *    Phi2 = 1/2) and F(b)(0, .) = 0, unless the regularised multiplier is
 *    chosen (kzk_params.reg_eps); at the tau-Nyquist index only the
 *    absorption part of l is kept.
 */
#ifndef KZK_H
#define KZK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kzk_plan kzk_plan;

typedef enum {
    KZK_OK = 0,
    KZK_ERR_ARG = 1,       /* invalid argument (null pointer, bad size, bad dtype, ...) */
    KZK_ERR_SIZE = 2,      /* grid size outside the supported range                      */
    KZK_ERR_OOM = 3,       /* device allocation failed                                   */
    KZK_ERR_DEVICE = 4,    /* a HIP call failed                                          */
    KZK_ERR_CFL = 5,       /* device: alpha * h / dtau exceeded cfl_max on some line     */
    KZK_ERR_NONFINITE = 6, /* device: NaN or Inf met in the field                        */
    KZK_ERR_STATE = 7      /* step range outside the coefficient schedule, or misuse     */
} kzk_status;

typedef enum { KZK_F32 = 0, KZK_F64 = 1 } kzk_dtype;

typedef struct {
    int32_t n_tau, n_y;     /* n_y a power of two in [16, 8192]; n_tau a power of two in
                               [32, 8192], or 7 * 2^k in [224, 7168] (the grids of Sec. 4,
                               N_theta = 7 * 2^k: a radix-7 stage in the tau-transform;
                               then every solve of the plan has the same n_tau).  With
                               n_y = 8192 the plan needs y-pass blocks of 512 or more
                               threads and full column tiles in every solve
                               (KZK_ERR_SIZE otherwise)                            */
    double tau0, L_tau;     /* periodic tau box [tau0, tau0 + L_tau)                      */
    double y0, L_y;         /* periodic y box [y0, y0 + L_y)                              */
    double x0, h;           /* marching origin and step: x_n = x0 + n h (paper: Delta sigma) */
    int32_t dtype;          /* kzk_dtype: arithmetic of every kernel; the multipliers are
                               always built in FP64 and stored in this precision           */
    double D;               /* diffraction (D/2) d_tau^{-1} d_yy, used when D_step == NULL */
    double A;               /* absorption A d_tau^2, A >= 0                                */
    double nl;              /* Burgers coefficient, used when nl_node == NULL              */
    const double *D_step;   /* optional host array [n_steps_max]: coefficient of step n,
                               e.g. the step average (1/h) int_{x_n}^{x_n+h} D(x) dx        */
    const double *nl_node;  /* optional host array [n_steps_max + 1]: nl(x_n); stage 1 of
                               step n uses nl(x_n), stage 2 uses nl(x_{n+1})                */
    int32_t n_steps_max;    /* length of the schedules (ignored when both are NULL)        */
    int32_t lf_scope;       /* 0: LF speed per tau-line (only value supported)             */
    double weno_eps;        /* WENO epsilon (> 0), 1e-6 in the usual reading               */
    double cfl_max;         /* alpha h / dtau above this latches KZK_ERR_CFL (0 -> 1.0)    */
    int32_t scheme;         /* 0: ExpRK22 (Sec. 3.3 eq. (19), Algorithm 2); 1: exponential
                               Euler, u^{n+1} = E u^n + h phi1(hL) b(x_n, u^n) (Sec. 3.3);
                               the same for every solve of a plan                           */
    double reg_eps;         /* 0: mean tau-mode zeroed (l = 0 there and F(b)(0, .) = 0);
                               > 0: the regularised multiplier of Sec. 3.4 (definition of
                               z_jk): 1/(i k_tau) becomes 1/(i k_tau + reg_eps / (4 pi)) at
                               every tau-mode, so the mean mode of every ky != 0 is damped
                               by exp(-h (D/2) ky^2 4 pi / reg_eps); the paper takes the
                               machine epsilon of the working precision                    */
    /* Transport by the random velocity field of Sec. 2 (Algorithm 1): b gains the
       terms 2 pi U_par d_tau u - U_perp d_y u of Sec. 3.3 eq. (16), taken in the
       conservative form of Sec. 3.4 eq. (21)-(22):
         b = -d_tau(nl u^2/2 - 2 pi U_par u) - d_y(U_perp u) + (d_y U_perp) u,
       WENO5/LF along tau (speed max |nl u - 2 pi U_par| per tau-line) and along y
       (speed max_j |U_perp|), with U evaluated at the stage nodes x_n, x_{n+1}.
       vel = 0: no transport; vel = 1: the field of vel_modes modes with phases
       vel_phi[n] and angles vel_theta[n] (host arrays, radians), r = vel_lambda (x, y),
       length scale L = 4 vel_lambda, |K_n| equispaced in [0.1/L, 9/L],
       |U~(K_n)| = sqrt(E(|K_n|)/N), E(K) = sigma_u^2 K^3 L^4 exp(-(K L/2)^2) / 8,
       normalised by vel_c0 (the paper: lambda = 6.86 m, sigma_u = 3 m/s,
       c0 = 343 m/s).  Needs 1 <= n_steps_max <= 65534 (the field is tabulated
       at the nodes 0 .. n_steps_max, with or without D_step / nl_node; steps
       beyond them return KZK_ERR_STATE); the same vel for every solve of a plan. */
    int32_t vel;
    int32_t vel_modes;
    const double *vel_phi, *vel_theta;
    double vel_lambda, vel_sigma_u, vel_c0;
    /* FP32 plans only (ignored in FP64): 1 keeps the spectral state U and the
       stage value P in FP64 (the combine of the y-passes in FP64, with the
       step's multipliers evaluated in FP64 in stage 1), everything else in
       FP32.  Without it the FP32 state is rounded every step while changing by
       about one unit of FP32 rounding per step (E is within a few rounding
       units of 1 at small h), so the rounding error adds up coherently over a
       march.  The same for every solve of a plan; not with reg_eps > 0. */
    int32_t state_fp64;
} kzk_params;

/* Create a plan for n_inst independent solves (n_inst >= 1), params[i] for
 * solve i; uneven grids are allowed.  Allocates the workspace, builds the
 * twiddle table and the E/Phi1/Phi2 multiplier tables (FP64 evaluation).
 * hip_stream: a hipStream_t, or NULL for the default stream.
 * Returns KZK_ERR_ARG / KZK_ERR_SIZE for invalid parameters, KZK_ERR_OOM
 * when device memory runs out, KZK_ERR_DEVICE for other HIP failures. */
kzk_status kzk_create(const kzk_params *params, int32_t n_inst, void *hip_stream, kzk_plan **out);

/* Advance the packed physical field u_dev (all solves, at the offsets of
 * kzk_inst_offset, in the plan's dtype) in place by n_steps ExpRK22 steps,
 * steps first_step .. first_step + n_steps - 1 (Algorithm 2, Sec. 4.2).
 * Asynchronous.  Deterministic: the same call on the same input gives the
 * same bits.  Running steps a..b then b..c equals running a..c up to one extra
 * tau-transform round trip of the field at b.
 * Returns KZK_ERR_STATE if the range leaves a given coefficient schedule. */
kzk_status kzk_step(kzk_plan *plan, void *u_dev, int32_t first_step, int32_t n_steps);

/* Discrete adjoint of kzk_step (transpose of the Jacobian of the whole
 * march, derived from Sec. 3.3 eq. (19)): given the field u0_dev at step
 * first_step and lam_dev = dL/du at step first_step + n_steps, write dL/du0
 * into grad_dev (may alias lam_dev).  The forward march is recomputed from
 * checkpoints taken every ckpt_every steps; the stage inputs of one interval
 * (2 ckpt_every fields) are stored, so ckpt_every >= n_steps recomputes
 * nothing.  ckpt_every = 0: the longest interval (halving from n_steps)
 * whose stored fields and checkpoints fit in half of the device memory free
 * at the call.  Asynchronous; the result does not depend on the interval.  For ExpRK22
 * with the mean mode zeroed and the Burgers b (scheme 0, reg_eps 0, vel 0,
 * state_fp64 0 in FP32), on every grid kzk_step takes; KZK_ERR_ARG
 * otherwise. */
kzk_status kzk_adjoint(kzk_plan *plan, const void *u0_dev, const void *lam_dev, int32_t first_step,
                       int32_t n_steps, int32_t ckpt_every, void *grad_dev);

/* Synchronise the plan's stream and return (and clear) the device status:
 * KZK_ERR_NONFINITE, then KZK_ERR_CFL, else KZK_OK; KZK_ERR_DEVICE if the
 * stream reports an error. */
kzk_status kzk_poll(kzk_plan *plan);

/* Element offset of solve i in the packed field buffer; the buffer holds
 * kzk_inst_offset(plan, n_inst) elements.  Returns (size_t)-1 for bad i. */
size_t kzk_inst_offset(const kzk_plan *plan, int32_t i);

/* Replace the HIP stream the plan enqueues on (NULL: default stream). */
kzk_status kzk_set_stream(kzk_plan *plan, void *hip_stream);

/* Enable (1) or disable (0) replay of kzk_step through a captured HIP graph.
 * The graph for one (u_dev, first_step, n_steps) is cached and reused.  The
 * legacy default stream cannot be captured: with graphs enabled, kzk_step on
 * a plan without a stream of its own (hip_stream NULL at kzk_create or
 * kzk_set_stream) returns KZK_ERR_STATE. */
kzk_status kzk_set_graph(kzk_plan *plan, int32_t enable);

/* Select the y-pass block size (256, 512 or 1024 threads; 1024 in FP32
 * only); rebuilds the tiled multiplier tables.  0 restores the default: the
 * smallest size whose column tiles are at least 32 bytes wide.  KZK_ERR_ARG
 * if 16 * threads < n_y of some solve; KZK_ERR_SIZE (plan unchanged) for a
 * size that leaves a solve with n_y = 8192 without full column tiles. */
kzk_status kzk_set_y_threads(kzk_plan *plan, int32_t threads);

/* Select the tau-pass block size: 256 threads (one 8192-point line per
 * block), or 512 in FP32 only (two such lines, so the rows that share the
 * 128-byte lines of the column-tiled spectra belong to fewer blocks);
 * 256 only with n_tau = 7 * 2^k.  0 restores the default (256). */
kzk_status kzk_set_tau_threads(kzk_plan *plan, int32_t threads);

/* Select the radix schedule of the power-of-two tau-transforms: 16
 * (radix-16 stages, then one radix-2/4/8 tail; the default) or 8 (radix-8
 * stages, then one radix-2/4 tail: one more LDS pass per transform, half the
 * values per butterfly in registers).  16 only with n_tau = 7 * 2^k.
 * 0 restores the default.  KZK_ERR_ARG for other values. */
kzk_status kzk_set_tau_fft_radix(kzk_plan *plan, int32_t radix);
int32_t kzk_get_tau_fft_radix(const kzk_plan *plan);

/* Autotuner: time n_trial steps on the plan's own scratch state (u_dev is
 * read, never written) for every supported combination of y-pass block
 * size, tau-pass block size and tau-transform radix schedule, keep the
 * fastest and return its y-pass block size (> 0), or -(kzk_status) on
 * error.  The y-pass block size fixes the column-tile width
 * W = threads * 16 / n_y of the y-FFTs and of the spectral layout (and so
 * the row segments of the tau-pass); the tau-pass block size fixes how many
 * tau-lines one block transforms and differentiates together.  If the
 * environment variable KZK_TUNE_CACHE names a file, a plan whose key (device
 * architecture, dtype, scheme, every solve's grid) is listed there takes the
 * stored choice without timing, and a timed result is appended to it as the
 * text line "<key> <y_threads> <tau_threads> <tau_fft_radix> <ms per step>".
 * Synchronises. */
int32_t kzk_autotune(kzk_plan *plan, const void *u_dev, int32_t n_trial);

/* Current y-pass block size. */
int32_t kzk_get_y_threads(const kzk_plan *plan);

/* Current tau-pass block size. */
int32_t kzk_get_tau_threads(const kzk_plan *plan);

/* Kernel classes reported by kzk_profile_read. */
enum {
    KZK_KIND_TAU = 0,        /* tau-pass: inverse tau-FFT, WENO5 b, forward tau-FFT      */
    KZK_KIND_Y1 = 1,         /* y-pass, stage 1 (y-FFTs, E/Phi1/Phi2 combine, inverse)    */
    KZK_KIND_Y2 = 2,         /* y-pass, stage 2                                          */
    KZK_KIND_TABLES = 3,     /* multiplier table build (FP64)                            */
    KZK_KIND_TRANSFORM = 4,  /* plain tau-transforms at the ends of a march              */
    KZK_KIND_ADJ_TAU = 5,    /* adjoint tau-pass (WENO5 Jacobian transpose)              */
    KZK_KIND_ADJ_Y = 6,      /* adjoint y-passes                                         */
    KZK_KIND_TRANSPORT = 7,  /* transverse transport pass (WENO5 along y, source)        */
    KZK_N_KINDS = 8
};

/* Bracket later kernel launches of the plan with HIP events on its stream:
 * every = 0 stops; every = k >= 1 brackets the launches of the forward steps
 * s with s % k == 0 and all other launches (k = 1: every launch).  While on,
 * graph replay is not used.  For measurement; an event record costs a few
 * microseconds of queue time, so sampling (k > 1) keeps the march it
 * measures close to an unprofiled one.  KZK_ERR_ARG for every < 0. */
kzk_status kzk_profile_enable(kzk_plan *plan, int32_t every);

/* Synchronise the stream and return, per kernel class k < n_kinds, the summed
 * event time ms[k] (milliseconds) and the number of launches count[k] since
 * the last read; then forget them. */
kzk_status kzk_profile_read(kzk_plan *plan, double *ms, int32_t *count, int32_t n_kinds);

/* Release the plan and its device memory (after finishing its stream work). */
void kzk_destroy(kzk_plan *plan);

const char *kzk_status_str(kzk_status s);

/* ---- march without device allocation ----
 * For callers that cannot allocate device memory (code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * kzk_step_noalloc(params, n_inst, hip_stream, u_dev, first_step, n_steps)
 * does what kzk_create + kzk_step + kzk_poll + kzk_destroy do, with the same
 * kernels and results, but takes all of its device memory (spectral state,
 * stage arrays, multiplier and twiddle tables, work lists, status word) from
 * one static device array of KZK_NOALLOC_SCRATCH_BYTES per GPU, which that
 * GPU holds from the library's load until the process ends.  It calls no
 * hipMalloc or hipFree.  Arguments as for kzk_create and kzk_step; u_dev is
 * caller-owned.  Returns KZK_ERR_SIZE when the solves do not fit the array
 * (about 2^20 grid points in FP32, 2^19 in FP64), the errors of kzk_create /
 * kzk_step for invalid arguments, else the device status (KZK_OK,
 * KZK_ERR_CFL or KZK_ERR_NONFINITE).  Synchronises the stream before it
 * returns.  Every call on one GPU uses that GPU's array and overwrites what
 * the last call left there: calls that overlap on one GPU (from several host
 * threads) race and must not be made. */
#define KZK_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
kzk_status kzk_step_noalloc(const kzk_params *params, int32_t n_inst, void *hip_stream, void *u_dev,
                            int32_t first_step, int32_t n_steps);

/* ---- single-operator entry points (used for per-kernel parity) ----
 * Each applies one piece of the step to every solve of the plan. */

/* b = -nl d_tau(u^2/2) by WENO5/LF on every tau-line of u_dev, with
 * nl = nl(x_node) (Sec. 3.4): b_dev receives the physical field b.  Runs the
 * production tau-pass kernel (which leaves the tau-spectrum of the face
 * fluxes) between a forward transform and, after the flux-difference
 * multiplier sigma_m = -(1 - e^{-2 pi i m / n_tau}) / dtau, an inverse one. */
kzk_status kzk_eval_b(kzk_plan *plan, const void *u_dev, int32_t node, void *b_dev);

/* Forward tau-transform of the physical field (R2C along tau, packed: slot 0
 * holds (X_0, X_{n_tau/2})) into spec_dev, M = n_tau/2 complex per row. */
kzk_status kzk_tau_forward(kzk_plan *plan, const void *u_dev, void *spec_dev);

/* Inverse of kzk_tau_forward (scaled by 1/n_tau). */
kzk_status kzk_tau_inverse(kzk_plan *plan, const void *spec_dev, void *u_dev);

/* Copy the multiplier tables of solve inst into out_dev (device buffer of
 * 3 * (n_tau/2) * (n_y/2 + 1) complex values of the plan's dtype), ordered
 * [table][m][n] for tau-mode m < n_tau/2 and |ky index| n <= n_y/2, tables
 * E/n_y, h Phi1/n_y, h Phi2/n_y of z = h l(m, n) (Sec. 3.4); entry (m = 0,
 * n = 0) holds the unscaled tau-Nyquist scalars e^z, h phi1(z), h phi2(z)
 * with z = -h A k_N^2, other m = 0 entries are zero.  Synchronises. */
kzk_status kzk_read_tables(kzk_plan *plan, int32_t inst, void *out_dev);

#ifdef __cplusplus
}
#endif
#endif
