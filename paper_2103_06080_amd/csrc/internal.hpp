// internal.hpp -- data shared by the host runtime and the kernels of libkzk.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kzk {

// Status bits latched by the kernels (vector atomics on a device word).
enum : unsigned { ST_CFL = 1u, ST_NONFINITE = 2u };

// A tau-line of n_tau reals is handled as a complex sequence of M = n_tau/2
// points by M/16 threads; a tau-pass block of nt threads holds nt*16 complex
// points, i.e. nt*32/n_tau lines: TAU_THREADS (256; FP64, the adjoint and the
// default) or TAU_THREADS_WIDE (512, FP32 only: two 8192-point lines, so the
// rows that share the 128-byte lines of the column-tiled spectra are written
// by fewer blocks, still two blocks per compute unit).
constexpr int TAU_THREADS = 256;
constexpr int TAU_THREADS_WIDE = 512;

// One solve of a (possibly batched) plan, as the kernels see it.
struct InstDesc {
    int n_tau, n_y;        // grid points along tau and y
    int M, Nh;             // M = n_tau/2 complex tau-modes (packed), Nh = n_y/2 + 1
    int W, log2W;          // y-pass tile width (columns per block)
    int rows_per_tau_block;  // lines per tau-pass block (threads * 16 / M)
    int scheme;              // 0: ExpRK22, 1: exponential Euler
    long long off_state;   // complex offset of this solve in the C, B, P arrays
    long long off_u;       // real offset of this solve in the packed physical field
    long long off_tab;     // complex offset in each multiplier table
    long long tab_size;    // M * Nh elements of this solve in each table
    long long tab_stride;  // distance between the E, Phi1 and Phi2 tables (all solves)
    double dtau, h, L_tau, L_y, A, weno_eps;
    double D_const, nl_const, cfl_max;
    double reg_eps;          // > 0: regularised multiplier, 1/(i kt) -> 1/(i kt + reg_eps/(4 pi))
    // transport by the random velocity field (vel = 1): per node x_n of the
    // schedule, vel_tab[n][0..2][j] = U_par, U_perp, d_y U_perp at y_j (FP64)
    // and vel_amax[n] = max_j |U_perp|, the LF speed along y
    int vel, pad1;
    double y0, dy;
    const double* vel_tab;
    const double* vel_amax;
    const double* nl_node;   // device [n_steps_max+1] or nullptr -> nl_const
    const double* D_step;    // device [n_steps_max]   or nullptr -> D_const
    // device [M] complex (working precision): flux-difference symbol sigma_m
    // = -(1 - e^{-2 pi i m / n_tau}) / dtau of tau-mode m (m = 0: zero)
    const void* sigma;
};

struct TauItem { int inst, row0; };
struct YItem { int inst, m0; };
// transverse WENO5 pass: 256 tau-points from k0, YW_SEG rows from j0
struct YwItem { int inst, k0, j0; };
constexpr int YW_SEG = 32;
constexpr int YW_THREADS = 256;

// Launchers (kernels.hip).  All enqueue on `s` and return hipSuccess or the
// launch error.  tw: twiddles exp(-2 pi i k / 2^log2_ntw); twst: per-stage
// Stockham twiddles of all transform lengths 2^4 .. 2^13 (fft.hpp).
// prog: every instance has M/16 >= W and M >= 256 (tiled spectra; enables
// progression indexing in the mode-2 kernel).
// nt: threads per block (tau_threads_supported).  gk > 0: every instance
// has M = 7 * 2^gk (4 <= gk <= 9), nt = TAU_THREADS, tw holds
// exp(-2 pi i k / n_tau) for k < n_tau, and twst, log2_ntw, prog and mr are
// unused.  mr: radix schedule of the power-of-two tau-transforms (log2 of the
// largest radix, 4 or 3).
template <typename T>
hipError_t launch_tau(int mode, int nt, const InstDesc* d_desc, const TauItem* d_items, int n_items, const T* u_in,
                      T* u_out, const void* Cin, void* Bout, const void* tw, const void* twst, int log2_ntw,
                      int node, int tiled, int prog, int gk, int mr, unsigned* status, hipStream_t s);
bool tau_threads_supported(int dtype_is_f64, int nt);

// y-pass over n_items column tiles with at most max_blocks persistent blocks
// (0: one block per tile).  step: index into the D schedule of instances
// whose multipliers the y-pass computes itself (those with D_step; stage 1
// then writes their h Phi2 table for stage 2).  full: 1 if every instance
// has W n_y = 16 nt and n_y >= 512 (full tiles; progression addressing), 2
// if so and some instance has n_y = 8192 (nt >= 512), else 0.
// By: tau-spectrum of the transverse transport part of b (instances with
// vel = 1; nullptr otherwise), added to sigma_m B before the y-transform.
// s64: an FP32 plan whose spectral state U and stage value P are FP64.
// ntl: full tiles with an FP64 state (FP64 plans, or s64) load U, P and the
// tables non-temporally (for arrays larger than the caches).
template <typename T>
hipError_t launch_y(int stage, int s64, int ntl, int nt, int full, const InstDesc* d_desc, const YItem* d_items,
                    int n_items, int max_blocks, void* C, const void* B, const void* By, void* P, void* U, void* tabs,
                    const void* twst, int step, hipStream_t s);

// Transverse part of b on the physical field u at node `node`:
// by = -(G_{j+1/2} - G_{j-1/2}) / dy + (d_y U_perp)_j u_j, G the WENO5/LF flux
// of g = U_perp u along y (instances with vel = 1).
template <typename T>
hipError_t launch_yweno(const InstDesc* d_desc, const YwItem* d_items, int n_items, const T* u, T* by, int node,
                        unsigned* status, hipStream_t s);

// Velocity tables of one instance for nodes 0 .. n_nodes-1 (FP64), from the
// per-mode wavenumber K_n lambda, amplitude, cos and sin of the angle, and
// phase (modes[5][n_modes]).
hipError_t launch_velocity(const InstDesc* d_desc, int inst, const double* modes, int n_modes, double x0, double h,
                           int n_nodes, double* tab, double* amax, hipStream_t s);
// blocks of the y-pass kernels (block size nt, full as for launch_y)
// resident at once on the device
int y_resident_blocks(int dtype_is_f64, int s64, int nt, int full, int device);

template <typename T>
hipError_t launch_tables(const InstDesc* d_desc, int inst, int per_tile, int n_tiles, void* tabs, int step,
                         hipStream_t s);

// b^ = sigma_m F^ (+ Y, the spectrum of the transverse transport part, when
// Y is not null) in place on instance inst's tiled tau-spectrum (n = M n_y
// elements): the flux difference applied to a tau-pass result.
template <typename T>
hipError_t launch_flux_diff(const InstDesc* d_desc, int inst, long long n, void* X, const void* Y, hipStream_t s);

// Mean tau-mode column of the regularised multiplier (instances with
// reg_eps > 0; one block per instance, the others return at once), after
// y-pass stage 1: C~*(0, .) = F_y^-1[E_0 U^ + h Phi1_0 b^], P(0, .) =
// F_y^-1[E_0 U^ + h (Phi1_0 - Phi2_0) b^]; after stage 2 (transport only):
// U(0, .) = C~(0, .) = P(0, .) + F_y^-1[h Phi2_0 b*^].  b^ is the y-transform
// of the mean of b (By column 0), zero without transport.
template <typename T>
hipError_t launch_dc(int stage, const InstDesc* d_desc, int n_inst, void* C, void* P, void* U, const void* By,
                     const void* twst, int step, hipStream_t s);

// gk as for launch_tau (M = 7 * 2^gk lines, tw of length n_tau).
template <typename T>
hipError_t launch_tau_adj(int stage, const InstDesc* d_desc, const TauItem* d_items, int n_items, const void* Tin,
                          const void* Rin, const T* ustore, void* out, const void* tw, const void* twst,
                          int log2_ntw, int node, int gk, unsigned* status, hipStream_t s);

// big: some instance has n_y = 8192 (nt 512, or 1024 in FP32).
template <typename T>
hipError_t launch_y_adj(int stage, int nt, bool big, const InstDesc* d_desc, const YItem* d_items, int n_items,
                        const void* In, void* Lh, void* Tout, void* Rout, const void* tabs, const void* twst,
                        hipStream_t s);

// Number of complex entries of the per-stage twiddle table (all lengths).
int stage_twiddle_entries();
// Fill it (FP64) in the layout of fft.hpp: for each length 2^LN (LN = 4..13),
// for each stage with Ns > 1, entries exp(-2 pi i k s / (Ns R)) at s*Ns + k.
void stage_twiddles(double* out_interleaved);

// Block sizes of the y-pass for which kernels are compiled.
bool y_threads_supported(int dtype_is_f64, int nt);

}  // namespace kzk
