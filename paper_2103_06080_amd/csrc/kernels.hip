// kernels.hip -- HIP kernels of the exponential-integrator/WENO5 step (gfx950).
//
// Spectra are packed R2C along tau: M = n_tau/2 complex per row, slot 0
// holds the real DC mode in .x and the real tau-Nyquist mode in .y.
//
// The state between steps is the full spectrum U = F(u) (as in Algorithm 2),
// with its tau-spectrum per y-row C~ (y physical) alongside for the next
// tau-pass.  One ExpRK22 step (Sec. 3.4 eq. (20), Algorithm 2) is four kernels:
//   tau-pass (node x_n)      C~  -> inverse tau-FFT -> u^n -> LF speed ->
//                                    WENO5 b -> forward tau-FFT -> B~
//   y-pass stage 1           y-FFT of B~, E/Phi1/Phi2 combine with U:
//                                    U* = E U + h Phi1 B,  P = E U + h (Phi1-Phi2) B,
//                                    inverse y-FFT of U* -> C~*, P kept
//   tau-pass (node x_{n+1})  C~* -> B~*
//   y-pass stage 2           U^{n+1} = P + h Phi2 B*, inverse y-FFT -> C~
// Column 0 (DC and tau-Nyquist) needs no y-FFT: the DC multipliers are
// (1, 1, 1/2) with F(b)(0, .) = 0, so the DC column is left untouched, and
// the Nyquist multipliers do not depend on ky, so they act pointwise in y.
#include "fft.hpp"
#include "internal.hpp"

#include <float.h>
#include <type_traits>

namespace kzk {

constexpr double KZK_PI = 3.14159265358979323846264338327950288;

template <typename T> struct alignas(4 * sizeof(T)) quad { T v[4]; };

// Four consecutive reals of a line buffer = two complex slots 2c, 2c+1 of
// the row starting at logical index base (base + 2c is even, so the pair
// never straddles a pad slot).
template <typename T> __device__ __forceinline__ quad<T> lds_quad(const cpx<T>* lds, int base, int c) {
    const int i = padi(base + 2 * c);
    cpx<T> a = lds[i], b = lds[i + 1];
    return quad<T>{{a.x, a.y, b.x, b.y}};
}
template <typename T> __device__ __forceinline__ void lds_quad_st(cpx<T>* lds, int base, int c, quad<T> q) {
    const int i = padi(base + 2 * c);
    lds[i] = cpx<T>{q.v[0], q.v[1]};
    lds[i + 1] = cpx<T>{q.v[2], q.v[3]};
}

template <typename T> __device__ __forceinline__ T rcp(T x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) {
    // hardware estimate refined by two Newton steps
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

template <typename T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
// complex value in another precision
template <typename S, typename T> __device__ __forceinline__ cpx<S> cvs(cpx<T> a) { return cpx<S>{(S)a.x, (S)a.y}; }
// maximum that propagates NaN (IEEE 754-2019 maximum; v_maximum3_f32 in FP32)
template <typename T> __device__ __forceinline__ T nmax(T a, T b) { return __builtin_elementwise_maximum(a, b); }

// Raw buffer access (gfx9 descriptor: 32-bit data format, no stride, no
// range limit below 2 GiB): a per-thread byte offset plus a wave-uniform byte
// offset, so that accesses at uniform strides need no per-access address
// arithmetic.  Every caller stays inside the array it addresses.  CP is the
// access's cache policy: 0, or CP_NT (the gfx950 non-temporal bit: the lines
// are not kept for reuse in L2 and the Infinity Cache).
constexpr int CP_NT = 2;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7fffffff, 0x00020000);
}
template <typename T, int CP = 0>
__device__ __forceinline__ cpx<T> buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP));
    } else {
        return __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, CP));
    }
}
template <typename T, int CP = 0>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, cpx<T> v) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, CP);
    } else {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, voff, soff, CP);
    }
}
// Non-temporal store of one complex value (plain addressing).
template <typename T>
__device__ __forceinline__ void st_nt(cpx<T>* p, cpx<T> v) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(__builtin_bit_cast(v2, v), reinterpret_cast<v2*>(p));
}
template <typename T> __device__ __forceinline__ bool finite_val(T x);
template <> __device__ __forceinline__ bool finite_val<float>(float x) { return fabsf(x) <= FLT_MAX; }
template <> __device__ __forceinline__ bool finite_val<double>(double x) { return fabs(x) <= DBL_MAX; }

// ------------------------------------------------------------------ WENO5-JS
// Face value from the upwind-ordered stencil v0..v4 (v2 on the upwind side of
// the face): candidates q_r, smoothness indicators beta_r (Jiang-Shu), ideal
// weights (1/10, 6/10, 3/10), p = 2.  The three nonlinear weights share one
// reciprocal: w_r ~ d_r prod_{s != r} (eps + beta_s)^2.
template <typename T>
__device__ __forceinline__ T weno_face(T v0, T v1, T v2, T v3, T v4, T eps) {
    const T c1312 = (T)(13.0 / 12.0);
    T q0 = (T)2 * v0 - (T)7 * v1 + (T)11 * v2;
    T q1 = -v1 + (T)5 * v2 + (T)2 * v3;
    T q2 = (T)2 * v2 + (T)5 * v3 - v4;
    T a0 = v0 - (T)2 * v1 + v2, b0 = v0 - (T)4 * v1 + (T)3 * v2;
    T a1 = v1 - (T)2 * v2 + v3, b1 = v1 - v3;
    T a2 = v2 - (T)2 * v3 + v4, b2 = (T)3 * v2 - (T)4 * v3 + v4;
    T s0 = eps + c1312 * a0 * a0 + (T)0.25 * b0 * b0;
    T s1 = eps + c1312 * a1 * a1 + (T)0.25 * b1 * b1;
    T s2 = eps + c1312 * a2 * a2 + (T)0.25 * b2 * b2;
    s0 *= s0; s1 *= s1; s2 *= s2;
    T w0 = (T)0.1 * s1 * s2, w1 = (T)0.6 * s0 * s2, w2 = (T)0.3 * s0 * s1;
    return (w0 * q0 + w1 * q1 + w2 * q2) * rcp((T)6 * (w0 + w1 + w2));
}

// WENO5-JS fluxes of one Lax-Friedrichs part at the eight faces 8g + k + 1/2
// (k < 8) from the points u[0..15] = u_{8g-4} .. u_{8g+11}; SIGN = +1 adds
// the reconstruction of f+ = (f + alpha u)/2 from the left, SIGN = -1 that of
// f- = (f - alpha u)/2 from the right, into F[k] (SIGN = +1 initialises it).
// The same values as weno_face, arranged so that work shared by adjacent
// faces is done once per point: with first differences d_j = f_{j+1} - f_j
// and second differences D_j = d_j - d_{j-1} of the split flux,
//   beta_r = 13/12 D^2 + 1/4 b_r^2 with b_r = D +- 2 d or d_{j-1} + d_j,
//   q_0 - q_1 = (D_{j-1} - D_j)/3,  q_2 - q_1 = (D_j - D_{j+1})/6,
// and the face value is q_1 + w_0 (q_0 - q_1) + w_2 (q_2 - q_1).  The code
// carries 4 (eps + beta_r) = 13/3 D^2 + b_r^2 + 4 eps, a power-of-two scaling
// common to the three weights (exact; the weights are unchanged).
template <typename T, int SIGN>
__device__ __forceinline__ void weno_group(const T (&u)[16], T nlq, T ha, T alpha, T eps, T (&F)[8]) {
    const T c133 = (T)(13.0 / 3.0), sixth = (T)(1.0 / 6.0), eps4 = (T)4 * eps;
    // split flux at the points 8g - 2 .. 8g + 10 (index j = point - 8g + 2)
    T f[13];
    #pragma unroll
    for (int j = 0; j < 13; ++j) {
        const T x = u[j + 2];
        const T fp = x * fma(nlq, x, ha);           // (nl u^2/2 + alpha u)/2
        f[j] = SIGN > 0 ? fp : fma(-alpha, x, fp);  // (nl u^2/2 - alpha u)/2
    }
    T dd[12], D2[12], A[12], G[12];
    #pragma unroll
    for (int j = 0; j < 12; ++j) dd[j] = f[j + 1] - f[j];
    #pragma unroll
    for (int j = 1; j < 12; ++j) {
        D2[j] = dd[j] - dd[j - 1];
        A[j] = fma(c133 * D2[j], D2[j], eps4);
    }
    #pragma unroll
    for (int j = 1; j < 11; ++j) G[j] = D2[j] - D2[j + 1];
    #pragma unroll
    for (int k = 0; k < 8; ++k) {
        // upwind point c, stencil neighbours a (upwind side) and b (downwind side)
        const int c = SIGN > 0 ? k + 2 : k + 3;
        const int a = c - SIGN, b = c + SIGN;
        // d between c and a / c and b, oriented along the stencil
        const T dca = SIGN > 0 ? dd[a] : -dd[c];     // f_c - f_a
        const T dbc = SIGN > 0 ? dd[c] : -dd[b];     // f_b - f_c
        const T b0 = fma((T)2, dca, D2[a]);
        const T b1 = dca + dbc;
        const T b2 = fma((T)-2, dbc, D2[b]);
        T s0 = fma(b0, b0, A[a]), s1 = fma(b1, b1, A[c]), s2 = fma(b2, b2, A[b]);
        s0 *= s0; s1 *= s1; s2 *= s2;
        const T t12 = s1 * s2, t02 = s0 * s2, t01 = s0 * s1;
        // 30 (0.1 t12 + 0.6 t02 + 0.3 t01)
        const T den = fma((T)3, t12, fma((T)18, t02, (T)9 * t01));
        // 30 [0.1 t12 (q0 - q1) + 0.3 t01 (q2 - q1)]
        const T Ga = SIGN > 0 ? G[a] : -G[c], Gc = SIGN > 0 ? G[c] : -G[b];
        const T num = fma(t12, Ga, t01 * ((T)1.5 * Gc));
        const T q1 = fma(sixth, fma((T)2, dbc, dca), f[c]);
        const T r = fma(num, rcp(den), q1);
        F[k] = SIGN > 0 ? r : F[k] + r;
    }
}

// ------------------------------------------------------------------ block helpers

// Max over the tpr threads of one line (lines are aligned groups of tpr
// consecutive threads; tpr is a power of two), NaN if any value is NaN.
// red: one LDS slot per wave.
template <typename T>
__device__ __forceinline__ T line_max(T v, int tpr, T* red) {
    const int w = tpr < 64 ? tpr : 64;
    for (int o = w >> 1; o > 0; o >>= 1) v = nmax(v, __shfl_xor(v, o));
    if (tpr > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = v;
        __syncthreads();
        const int nw = tpr >> 6, first = (threadIdx.x / tpr) * nw;
        T m = red[first];
        for (int i = 1; i < nw; ++i) m = nmax(m, red[first + i]);
        v = m;
        __syncthreads();
    }
    return v;
}

__device__ __forceinline__ int line_or(int v, int tpr, int* red) {
    const int w = tpr < 64 ? tpr : 64;
    for (int o = w >> 1; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    if (tpr > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = v;
        __syncthreads();
        const int nw = tpr >> 6, first = (threadIdx.x / tpr) * nw;
        int m = 0;
        for (int i = 0; i < nw; ++i) m |= red[first + i];
        v = m;
        __syncthreads();
    }
    return v;
}

// Block index -> work item so that items with consecutive indices run on the
// same XCD (blocks are dispatched round-robin over the 8 XCDs): neighbouring
// column tiles share cache lines of the row-major spectra.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// ------------------------------------------------------------------ tau-pass
// Real <-> packed half-spectrum along tau, using one complex FFT of M = N/2
// points: z_j = u_{2j} + i u_{2j+1}.
//
// Inverse (C2R), for the pair k, M-k (k = 0..M/2), scaled by 1/N:
//   A = X_k + conj X_{M-k},  P = i e^{+2 pi i k/N} (X_k - conj X_{M-k}),
//   Z_k = A + P,  Z_{M-k} = conj(A - P)
// Forward (R2C) from Z = FFT(z):
//   A = (Z_k + conj Z_{M-k})/2,  Q = i e^{-2 pi i k/N} (Z_k - conj Z_{M-k})/2,
//   X_k = A - Q,  X_{M-k} = conj(A + Q),  slot 0 = (X_0, X_M).

// Position of tau-mode k of one row in a spectral array: row-major rows of M
// modes, or column tiles [k / W][y][k % W] (tile = W modes x n_y rows).
// 32-bit arithmetic: within one instance every offset is below M n_y <= 2^24,
// so the tile product fits a 24-bit multiply.
struct SpecIdx {
    int lw;              // log2 W (tiles); 30 for row-major (k >> 30 = 0)
    unsigned mask;       // W - 1 (tiles); all ones below bit 30 for row-major
    unsigned stride;     // n_y * W (tiles); 0 for row-major
    __device__ __forceinline__ unsigned operator()(int k) const {
        return __umul24((unsigned)k >> lw, stride) + ((unsigned)k & mask);
    }
};
__device__ __forceinline__ SpecIdx spec_idx(int log2W, int n_y, bool tiled) {
    return tiled ? SpecIdx{log2W, (1u << log2W) - 1u, (unsigned)n_y << log2W} : SpecIdx{30, (1u << 30) - 1u, 0u};
}

// Positions of the pair (k, M - k), k = min(t + q*tpr, M/2), in a spectral
// row: X index of k, of (M - k) mod M, and twiddle index k << sh.
struct PairIdx {
    int t, tpr, M, sh;
    SpecIdx ix;
    __device__ __forceinline__ unsigned xk(int q) const { return ix(min(t + q * tpr, M >> 1)); }
    __device__ __forceinline__ unsigned xm(int q) const { return ix((M - min(t + q * tpr, M >> 1)) & (M - 1)); }
    __device__ __forceinline__ unsigned w(int q) const { return (unsigned)min(t + q * tpr, M >> 1) << sh; }
};

// One pair of the inverse: from X_k, X_{M-k} and the twiddle e^{-2 pi i k/N},
// Z_k and Z_{M-k} (both scaled by inv_n).
template <typename T>
__device__ __forceinline__ void c2r_pair(cpx<T> xk, cpx<T> xm, cpx<T> w, T inv_n, cpx<T>& zk, cpx<T>& zm) {
    const cpx<T> A = {xk.x + xm.x, xk.y - xm.y};
    const cpx<T> D = {xk.x - xm.x, xk.y + xm.y};
    const cpx<T> P = mul_si<1>(cmul(conj(w), D));    // i e^{+2 pi i k/N} D
    zk = inv_n * (A + P);
    zm = inv_n * conj(A - P);
}
// One pair of the forward: X_k and X_{M-k} from Z_k, Z_{M-k}.
template <typename T>
__device__ __forceinline__ void r2c_pair(cpx<T> zk, cpx<T> zm, cpx<T> w, cpx<T>& xk, cpx<T>& xm) {
    const cpx<T> A = {(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
    const cpx<T> D = {(T)0.5 * (zk.x - zm.x), (T)0.5 * (zk.y + zm.y)};
    const cpx<T> Q = mul_si<1>(cmul(w, D));          // i e^{-2 pi i k/N} D
    xk = A - Q;
    xm = conj(A + Q);
}

template <typename T>
__device__ __forceinline__ void c2r_pre(const cpx<T>* __restrict__ X, SpecIdx ix, cpx<T>* lds, int base, int M, int t,
                                        int tpr, const cpx<T>* __restrict__ tw, int log2_ntw, T inv_n) {
    // pairs k = t + q*tpr <= M/2, q < 9 (tpr = M/16); all loads of the thread are
    // issued before any is used, so their latencies overlap
    const int sh = log2_ntw - ilog2(2 * M);
    constexpr int Q = 9;
    const PairIdx pi{t, tpr, M, sh, ix};
    cpx<T> xk[Q], xm[Q], wv[Q];
    #pragma unroll
    for (int q = 0; q < Q; ++q) {
        xk[q] = X[pi.xk(q)];
        xm[q] = X[pi.xm(q)];
        wv[q] = tw[pi.w(q)];
    }
    #pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = t + q * tpr;
        if (k > (M >> 1)) continue;
        if (k == 0) {
            const cpx<T> s = xk[q];
            lds[padi(base)] = cpx<T>{(s.x + s.y) * inv_n, (s.x - s.y) * inv_n};
            continue;
        }
        cpx<T> zk, zm;
        c2r_pair(xk[q], xm[q], wv[q], inv_n, zk, zm);
        lds[padi(base + k)] = zk;
        if (2 * k != M) lds[padi(base + M - k)] = zm;
    }
}

// add: a spectrum in the same layout added to the result (nullptr: none).
template <typename T>
__device__ __forceinline__ void r2c_post(const cpx<T>* lds, int base, cpx<T>* __restrict__ X, SpecIdx ix, int M, int t,
                                         int tpr, const cpx<T>* __restrict__ tw, int log2_ntw,
                                         const cpx<T>* __restrict__ add = nullptr) {
    const int sh = log2_ntw - ilog2(2 * M);
    const PairIdx pi{t, tpr, M, sh, ix};
    #pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int k = t + q * tpr;
        if (k > (M >> 1)) continue;
        const cpx<T> zk = lds[padi(base + k)];
        const cpx<T> zm = lds[padi(base + ((M - k) & (M - 1)))];
        cpx<T> a, b;
        r2c_pair(zk, zm, tw[pi.w(q)], a, b);
        if (k == 0) {
            a = cpx<T>{a.x, b.x};   // slot 0 = (X_0, X_M) = (A - Q, A + Q) real parts
            X[0] = add ? a + add[0] : a;
            continue;
        }
        X[pi.xk(q)] = add ? a + add[pi.xk(q)] : a;
        if (2 * k != M) X[pi.xm(q)] = add ? b + add[pi.xm(q)] : b;
    }
}

// The same two for tiled spectra with W <= tpr = M/16 and tpr a multiple of
// 16 (M >= 256).  For q < 8 the pair k = t + q tpr lies in [0, M/2); from one
// q to the next its tile position, that of M - k and its twiddle index move
// by wave-uniform steps (whole tiles), and so do the padded LDS slots of k
// and M - k (16-aligned strides).  The global accesses are buffer accesses
// with a per-thread base and a uniform offset, the LDS ones a per-thread
// base plus a uniform offset; k = 0 (t = 0, q = 0) is a select and
// k = M/2 (t = 0 only) is done apart.  X: the instance's array (a
// block-uniform address, so the buffer descriptor stays in scalar
// registers), ro: the row's element offset in it.
template <typename T>
__device__ __forceinline__ void c2r_pre_prog(const cpx<T>* X, unsigned ro, SpecIdx ix, cpx<T>* lds, int base, int M,
                                             int t, int tpr, const cpx<T>* tw, int log2_ntw, T inv_n) {
    constexpr unsigned E = sizeof(cpx<T>);
    const int sh = log2_ntw - ilog2(2 * M);
    const unsigned step = __umul24((unsigned)tpr >> ix.lw, ix.stride) * E;   // bytes per q
    const unsigned wstep = ((unsigned)tpr << sh) * E;
    const unsigned k0 = (ro + ix(t)) * E;                // k at q = 0
    const unsigned m7 = (ro + ix(M - t - 7 * tpr)) * E;  // M - k at q = 7
    const unsigned w0 = ((unsigned)t << sh) * E;
    const auto xr = buf_rsrc(X), wr = buf_rsrc(tw);
    cpx<T> xk[8], xm[8], wv[8];
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        xk[q] = buf_ld<T>(xr, k0, q * step);
        // at q = 0, M - k = M for t = 0 lies outside the row: read X_0 there
        xm[q] = q == 0 ? buf_ld<T>(xr, t == 0 ? k0 : m7 + 7 * step, 0) : buf_ld<T>(xr, m7, (7 - q) * step);
        wv[q] = buf_ld<T>(wr, w0, q * wstep);
    }
    const int t17 = tpr + (tpr >> 4);
    const int pk = padi(base + t), pm = padi(base + M - t);
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        cpx<T> zk, zm;
        c2r_pair(xk[q], xm[q], wv[q], inv_n, zk, zm);
        if (q == 0 && t == 0) zk = cpx<T>{(xk[0].x + xk[0].y) * inv_n, (xk[0].x - xk[0].y) * inv_n};
        lds[pk + q * t17] = zk;
        if (q > 0 || t != 0) lds[pm - q * t17] = zm;
    }
    if (t == 0) {
        // k = M/2 pairs with itself
        const cpx<T> x = X[ro + ix(M >> 1)];
        cpx<T> zk, zm;
        c2r_pair(x, x, tw[(unsigned)(M >> 1) << sh], inv_n, zk, zm);
        lds[padi(base + (M >> 1))] = zk;
    }
}

template <typename T>
__device__ __forceinline__ void r2c_post_prog(const cpx<T>* lds, int base, cpx<T>* X, unsigned ro, SpecIdx ix, int M,
                                              int t, int tpr, const cpx<T>* tw, int log2_ntw) {
    constexpr unsigned E = sizeof(cpx<T>);
    const int sh = log2_ntw - ilog2(2 * M);
    const unsigned step = __umul24((unsigned)tpr >> ix.lw, ix.stride) * E;
    const unsigned wstep = ((unsigned)tpr << sh) * E;
    const unsigned k0 = (ro + ix(t)) * E;
    const unsigned m7 = (ro + ix(M - t - 7 * tpr)) * E;
    const unsigned w0 = ((unsigned)t << sh) * E;
    const auto xr = buf_rsrc(X), wr = buf_rsrc(tw);
    cpx<T> wv[8];
    #pragma unroll
    for (int q = 0; q < 8; ++q) wv[q] = buf_ld<T>(wr, w0, q * wstep);
    const int t17 = tpr + (tpr >> 4);
    const int pk = padi(base + t), pm = padi(base + M - t);
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        const cpx<T> zk = lds[pk + q * t17];
        const cpx<T> zm = lds[q == 0 ? (t == 0 ? pk : pm) : pm - q * t17];   // (M - k) mod M
        cpx<T> a, b;
        r2c_pair(zk, zm, wv[q], a, b);
        if (q == 0 && t == 0) a = cpx<T>{a.x, b.x};   // slot 0 = (X_0, X_M)
        buf_st<T>(xr, k0, q * step, a);
        // at q = 0, M - k = M for t = 0 lies outside the row: that thread
        // stores slot 0 a second time instead (same address, same value)
        if (q == 0) buf_st<T>(xr, t == 0 ? k0 : m7 + 7 * step, 0, t == 0 ? a : b);
        else buf_st<T>(xr, m7, (7 - q) * step, b);
    }
    if (t == 0) {
        const cpx<T> z = lds[padi(base + (M >> 1))];
        cpx<T> a, b;
        r2c_pair(z, z, tw[(unsigned)(M >> 1) << sh], a, b);
        X[ro + ix(M >> 1)] = a;
    }
}

// The two for M = 7 * 2^K (compile-time M): the same pairs k = t + q M/16
// (q < 9, k <= M/2), with M - k taken mod M by a select and the twiddle
// e^{-2 pi i k/N} read from the table tw[i] = e^{-2 pi i i/N} (N = 2M) at k.
template <typename T, int M>
__device__ __forceinline__ void c2r_pre_gen(const cpx<T>* __restrict__ X, SpecIdx ix, cpx<T>* lds, int base, int t,
                                            const cpx<T>* __restrict__ tw, T inv_n) {
    constexpr int tpr = M / 16, Q = 9;
    cpx<T> xk[Q], xm[Q], wv[Q];
    #pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = min(t + q * tpr, M / 2);
        xk[q] = X[ix(k)];
        xm[q] = X[ix(k == 0 ? 0 : M - k)];
        wv[q] = tw[k];
    }
    #pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = t + q * tpr;
        if (k > M / 2) continue;
        if (k == 0) {
            const cpx<T> s = xk[q];
            lds[padi(base)] = cpx<T>{(s.x + s.y) * inv_n, (s.x - s.y) * inv_n};
            continue;
        }
        cpx<T> zk, zm;
        c2r_pair(xk[q], xm[q], wv[q], inv_n, zk, zm);
        lds[padi(base + k)] = zk;
        if (2 * k != M) lds[padi(base + M - k)] = zm;
    }
}

template <typename T, int M>
__device__ __forceinline__ void r2c_post_gen(const cpx<T>* lds, int base, cpx<T>* __restrict__ X, SpecIdx ix, int t,
                                             const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ add = nullptr) {
    constexpr int tpr = M / 16;
    #pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int k = t + q * tpr;
        if (k > M / 2) continue;
        const cpx<T> zk = lds[padi(base + k)];
        const cpx<T> zm = lds[padi(base + (k == 0 ? 0 : M - k))];
        cpx<T> a, b;
        r2c_pair(zk, zm, tw[k], a, b);
        if (k == 0) {
            a = cpx<T>{a.x, b.x};
            X[0] = add ? a + add[0] : a;
            continue;
        }
        X[ix(k)] = add ? a + add[ix(k)] : a;
        if (2 * k != M) X[ix(M - k)] = add ? b + add[ix(M - k)] : b;
    }
}

// MODE 0: u -> C (R2C).  MODE 1: C -> u (C2R).  MODE 2: C -> B, the
// tau-spectrum of the WENO5 face fluxes F_{i+1/2} (the flux difference
// b_i = -(F_{i+1/2} - F_{i-1/2}) / dtau is the Fourier multiplier
// sigma_m = -(1 - e^{-2 pi i m / n_tau}) / dtau, applied by the y-pass).
// MODE 3: as MODE 2, and also stores the physical line u (for the adjoint).
// PROG (mode 2 only): tiled spectra with tpr a multiple of the tile width and
// of 16 in every instance (progression indexing of the pre/post-processing
// pairs).  NTT: threads per block; a block holds NTT * 16 complex points, the
// lines rows0 .. rows0 + NTT * 16 / M - 1.  GK > 0: every instance has
// M = 7 * 2^GK (n_tau = 7 * 2^(GK+1)); its M/16 threads per line sit in an
// aligned group of 2^(GK-1) (the rest of the group idle), so the block holds
// NTT / 2^(GK-1) lines, and tw is the table e^{-2 pi i k / n_tau}, k < n_tau.
// MR: radix schedule of the power-of-two transforms (4: radix 16, 3: radix 8).
template <typename T, int MODE, bool PROG = false, int NTT = TAU_THREADS, int GK = 0, int MR = 4>
__global__ __launch_bounds__(NTT) void tau_kernel(const InstDesc* __restrict__ descs,
                                                  const TauItem* __restrict__ items,
                                                  const T* __restrict__ u_in, T* __restrict__ u_out,
                                                  const cpx<T>* __restrict__ Cin, cpx<T>* __restrict__ Bout,
                                                  const cpx<T>* __restrict__ tw,
                                                  const cpx<T>* __restrict__ twst, int log2_ntw, int node,
                                                  int tiled, unsigned* __restrict__ status) {
    __shared__ alignas(32) cpx<T> lds[padded(NTT * 16)];
    __shared__ T redT[NTT / 64];
    __shared__ int redI[NTT / 64];
    // consecutive rows on one XCD: with column tiles, rows y..y+W-1 share cache lines
    const TauItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const InstDesc& d = descs[it.inst];
    static_assert(GK == 0 || (!PROG && NTT == TAU_THREADS), "lengths 7 * 2^K: plain indexing, 256 threads");
    const int M = GK ? (7 << GK) : d.M, N = 2 * M;
    const int tpr = M >> 4;
    const int tpg = GK ? (1 << (GK - 1)) : tpr;   // threads of a line's group (a power of two)
    const int r = threadIdx.x / tpg, t = threadIdx.x & (tpg - 1);
    const int row = it.row0 + r;
    const bool active = (GK == 0 || t < tpr) && (r < d.rows_per_tau_block) && (row < d.n_y);
    const int base = r * M;
    const int Nc = M >> 1;   // chunks of 4 reals per line
    const SpecIdx ix = spec_idx(d.log2W, d.n_y, tiled != 0);
    const long long so = d.off_state + (tiled ? ((long long)row << d.log2W) : (long long)row * M);

    if (MODE == 0) {
        const quad<T>* ug = reinterpret_cast<const quad<T>*>(u_in + d.off_u + (long long)row * N);
        int bad = 0;
        if (active) {
            quad<T> v[8];
            #pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = ug[t + q * tpr];
            #pragma unroll
            for (int q = 0; q < 8; ++q) {
                bad |= !(finite_val(v[q].v[0]) && finite_val(v[q].v[1]) && finite_val(v[q].v[2]) &&
                         finite_val(v[q].v[3]));
                lds_quad_st(lds, base, t + q * tpr, v[q]);
            }
        }
        bad = line_or(bad, tpg, redI);
        if (active && t == 0 && bad) atomicOr(status, ST_NONFINITE);
        __syncthreads();
        if constexpr (GK > 0) {
            gen_fft<T, -1, GK>(lds, base, t, active, tw);
            if (active) r2c_post_gen<T, (7 << GK)>(lds, base, Bout + so, ix, t, tw);
        } else {
            lds_fft<T, -1, true, MR>(lds, base, M, t, active, twst);
            if (active) r2c_post(lds, base, Bout + so, ix, M, t, tpr, tw, log2_ntw);
        }
        return;
    }

    // inverse tau-transform of C~ into the line buffer
    if (active) {
        if constexpr (GK > 0) c2r_pre_gen<T, (7 << GK)>(Cin + so, ix, lds, base, t, tw, (T)1 / (T)N);
        else if constexpr (PROG) c2r_pre_prog(Cin + d.off_state, (unsigned)row << d.log2W, ix, lds, base, M, t, tpr,
                                              tw, log2_ntw, (T)1 / (T)N);
        else c2r_pre(Cin + so, ix, lds, base, M, t, tpr, tw, log2_ntw, (T)1 / (T)N);
    }
    __syncthreads();
    if constexpr (GK > 0) gen_fft<T, 1, GK>(lds, base, t, active, tw);
    else lds_fft<T, 1, true, MR>(lds, base, M, t, active, twst);

    if (MODE == 1 || MODE == 3) {
        quad<T>* ug = reinterpret_cast<quad<T>*>(u_out + d.off_u + (long long)row * N);
        if (active) {
            #pragma unroll
            for (int q = 0; q < 8; ++q) ug[t + q * tpr] = lds_quad(lds, base, t + q * tpr);
        }
        if (MODE == 1) return;
    }

    // ---- LF speed alpha = |nl(x_node)| max|u| over the line (exact in any precision);
    // the maximum propagates NaN and Inf, so it also flags a non-finite line
    T mx = 0;
    if (active) {
        #pragma unroll
        for (int q = 0; q < 8; ++q) {
            const quad<T> v = lds_quad(lds, base, t + q * tpr);
            #pragma unroll
            for (int i = 0; i < 4; ++i) mx = nmax(mx, (T)fabs(v.v[i]));
        }
    }
    mx = line_max(mx, tpg, redT);
    bool bad = !finite_val(mx);
    const double nl = d.nl_node ? d.nl_node[node] : d.nl_const;
    const T nlT = (T)nl;
    T alpha = (T)fabs(nl) * mx;
    // transport: the tau-flux is nl u^2/2 - c u with c = 2 pi U_par(x_node, y_row),
    // so f' = nl u - c and alpha = max_k |nl u_k - c| = max(|nl max u - c|, |nl min u - c|)
    T cpar = 0;
    if (d.vel) {
        cpar = (T)(2.0 * KZK_PI * d.vel_tab[(size_t)node * 3 * d.n_y + (row < d.n_y ? row : 0)]);
        T hi = -mx, lo = -mx;             // max u and max(-u), NaN-propagating like mx
        if (active) {
            #pragma unroll
            for (int q = 0; q < 8; ++q) {
                const quad<T> v = lds_quad(lds, base, t + q * tpr);
                #pragma unroll
                for (int i = 0; i < 4; ++i) {
                    hi = nmax(hi, v.v[i]);
                    lo = nmax(lo, -v.v[i]);
                }
            }
        }
        hi = line_max(hi, tpg, redT);
        lo = line_max(lo, tpg, redT);
        alpha = tmax((T)fabs(nlT * hi - cpar), (T)fabs(nlT * -lo - cpar));
        bad = bad || !finite_val(alpha);
    }
    if (active && t == 0) {
        unsigned f = 0;
        if (bad) f |= ST_NONFINITE;
        if ((double)alpha * d.h > d.cfl_max * d.dtau) f |= ST_CFL;
        if (f) atomicOr(status, f);
    }

    // ---- WENO5 fluxes at the faces 8g + k + 1/2 (k < 8) of my groups g = t + q*tpr (q < 4)
    const T eps = (T)d.weno_eps;
    // split fluxes f+- = (nl u^2/2 - c u +- alpha u)/2 = u (nl u/4 + (+-alpha - c)/2)
    const T nlq = (T)0.25 * nlT, ha = (T)0.5 * (alpha - cpar);
    T F[4][8];
    #pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int g = t + q * tpr;
        if (active) {
            // points 8g - 4 .. 8g + 11
            T u[16];
            #pragma unroll
            for (int h = 0; h < 4; ++h) {
                int c = 2 * g - 1 + h;   // chunk index mod Nc
                if constexpr (GK > 0) c = c < 0 ? c + Nc : (c >= Nc ? c - Nc : c);
                else c &= Nc - 1;
                const quad<T> v = lds_quad(lds, base, c);
                #pragma unroll
                for (int i = 0; i < 4; ++i) u[4 * h + i] = v.v[i];
            }
            weno_group<T, 1>(u, nlq, ha, alpha, eps, F[q]);
            weno_group<T, -1>(u, nlq, ha, alpha, eps, F[q]);
        }
    }
    __syncthreads();
    #pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int g = t + q * tpr;
        if (active) {
            lds_quad_st(lds, base, 2 * g, quad<T>{{F[q][0], F[q][1], F[q][2], F[q][3]}});
            lds_quad_st(lds, base, 2 * g + 1, quad<T>{{F[q][4], F[q][5], F[q][6], F[q][7]}});
        }
    }
    __syncthreads();
    if constexpr (GK > 0) {
        gen_fft<T, -1, GK>(lds, base, t, active, tw);
        if (active) r2c_post_gen<T, (7 << GK)>(lds, base, Bout + so, ix, t, tw);
    } else {
        lds_fft<T, -1, true, MR>(lds, base, M, t, active, twst);
        if (active) {
            if constexpr (PROG) r2c_post_prog(lds, base, Bout + d.off_state, (unsigned)row << d.log2W, ix, M, t, tpr,
                                              tw, log2_ntw);
            else r2c_post(lds, base, Bout + so, ix, M, t, tpr, tw, log2_ntw);
        }
    }
}

// ------------------------------------------------------------------ multiplier tables
// phi-functions in FP64: Taylor series of phi2 (Horner) for |z| < 1, with
// phi1 = 1 + z phi2 and e^z = 1 + z phi1; closed forms otherwise.
// phi2 = sum_j z^j / (j+2)!; for |z| < 1 the terms beyond j = 17 add less
// than 1/20! relative to phi2 ~ 1/2, far below the FP64 rounding unit.
__host__ __device__ constexpr double inv_fact_plus2(int j) {
    double f = 1.0;
    for (int i = 2; i <= j + 2; ++i) f *= (double)i;
    return 1.0 / f;
}
// Closed forms (|z| >= 1).  Not inlined: the exponential and sine/cosine
// need many registers, and keeping them out of line keeps them out of the
// register allocation of the kernels that evaluate multipliers per mode
// (|z| >= 1 holds for few modes).
__device__ __attribute__((noinline)) void phis_closed_f64(double zr, double zi, cpx<double>& e, cpx<double>& p1,
                                                          cpx<double>& p2) {
    const cpx<double> z = {zr, zi};
    double ex = exp(zr), sn, cs;
    sincos(zi, &sn, &cs);
    e = {ex * cs, ex * sn};
    const double inv = 1.0 / (zr * zr + zi * zi);
    cpx<double> em1 = {e.x - 1.0, e.y};
    p1 = inv * cmulc(em1, z);                 // (e^z - 1) / z
    cpx<double> p1m1 = {p1.x - 1.0, p1.y};
    p2 = inv * cmulc(p1m1, z);                // (phi1 - 1) / z
}

__device__ void phis_f64(double zr, double zi, cpx<double>& e, cpx<double>& p1, cpx<double>& p2) {
    const cpx<double> z = {zr, zi};
    if (zr * zr + zi * zi < 1.0) {
        constexpr int J = 17;
        cpx<double> p = {inv_fact_plus2(J), 0.0};
        #pragma unroll
        for (int j = J - 1; j >= 0; --j) {
            p = cmul(z, p);
            p.x += inv_fact_plus2(j);
        }
        p2 = p;
        p1 = cmul(z, p2);
        p1.x += 1.0;
        e = cmul(z, p1);
        e.x += 1.0;
        return;
    }
    phis_closed_f64(zr, zi, e, p1, p2);
}

// z = h l of the regularised multiplier (Sec. 3.4, definition of z_jk):
// l = -(Dbar/2) ky^2 / (i kt + delta) - A kt^2, delta = eps / (4 pi),
//   = (Dbar/2) ky^2 (i kt - delta) / (kt^2 + delta^2) - A kt^2.
__device__ __attribute__((noinline)) void regularised_z(double eps, double A, double Dbar, double h, double kt,
                                                        double ky, double& zr, double& zi) {
    const double dl = eps / (4.0 * KZK_PI);
    const double q = 0.5 * Dbar * ky * ky / (kt * kt + dl * dl);
    zr = h * (-A * kt * kt - q * dl);
    zi = h * q * kt;
}

// Flux-difference symbol of tau-mode m (the table built at create, see
// InstDesc::sigma): the spectrum of b_i = -(F_{i+1/2} - F_{i-1/2}) / dtau is
// sigma_m times that of F_{i+1/2}.
template <typename T>
__device__ __forceinline__ cpx<T> flux_diff_symbol(const InstDesc& d, int m) {
    return static_cast<const cpx<T>*>(d.sigma)[m];
}

// Multipliers of mode (m, n) for step `step` (tau-mode m >= 1, |ky index| n),
// scaled by 1/n_y for the inverse y-transform: E/n_y, h Phi1/n_y, h Phi2/n_y.
template <typename T>
__device__ __forceinline__ void mode_multipliers(const InstDesc& d, int m, int n, int step, cpx<T>& E, cpx<T>& P1,
                                                 cpx<T>& P2) {
    const double h = d.h;
    const double Dbar = d.D_step ? d.D_step[step] : d.D_const;
    const double kt = 2.0 * KZK_PI * (double)m / d.L_tau;
    const double ky = 2.0 * KZK_PI * (double)n / d.L_y;
    // z = h l,  l = i Dbar ky^2 / (2 kt) - A kt^2 (the regularised symbol out of
    // line, so that it adds nothing to the registers of the unrolled per-mode code)
    double zr, zi;
    if (d.reg_eps > 0.0) {
        regularised_z(d.reg_eps, d.A, Dbar, h, kt, ky, zr, zi);
    } else {
        zr = -h * d.A * kt * kt;
        zi = h * Dbar * ky * ky / (2.0 * kt);
    }
    cpx<double> e, p1, p2;
    phis_f64(zr, zi, e, p1, p2);
    const double s = 1.0 / (double)d.n_y;
    E = cpx<T>{(T)(e.x * s), (T)(e.y * s)};
    P1 = cpx<T>{(T)(h * s * p1.x), (T)(h * s * p1.y)};
    P2 = cpx<T>{(T)(h * s * p2.x), (T)(h * s * p2.y)};
}

// The tau-Nyquist scalars (absorption only, ky-independent, not scaled).
template <typename T>
__device__ __forceinline__ void nyquist_multipliers(const InstDesc& d, T& E, T& P1, T& P2) {
    const double h = d.h;
    const double kn = 2.0 * KZK_PI * (double)(-d.M) / d.L_tau;
    cpx<double> e, p1, p2;
    phis_f64(-h * d.A * kn * kn, 0.0, e, p1, p2);
    E = (T)e.x;
    P1 = (T)(h * p1.x);
    P2 = (T)(h * p2.x);
}

// ------------------------------------------------------------------ transverse transport (Sec. 3.4 eq. (21)-(22))
// by_j = -(G_{j+1/2} - G_{j-1/2}) / dy + (d_y U_perp)_j u_j along every y-line
// of the physical field u, G the WENO5-JS flux with Lax-Friedrichs splitting
// of g_j = U_perp(x_node, y_j) u_j, speed alpha = max_j |U_perp| (g' does not
// depend on u): G = F+ + F-, F+ from g+ = (g + alpha u)/2 on rows j-2..j+2,
// F- from g- = (g - alpha u)/2 on the mirrored rows j+3..j-1.  A block of
// YW_THREADS threads takes YW_THREADS consecutive tau-points (one column
// each, coalesced) and YW_SEG rows from j0; it stages the rows j0-3 ..
// j0+YW_SEG+2 of its columns (periodic in y) in LDS, then each thread sweeps
// its column computing every face once.
template <typename T>
__global__ __launch_bounds__(YW_THREADS) void yweno_kernel(const InstDesc* __restrict__ descs,
                                                           const YwItem* __restrict__ items, const T* __restrict__ u,
                                                           T* __restrict__ by, int node, unsigned* __restrict__ status) {
    constexpr int R = YW_SEG + 6;
    __shared__ T us[R][YW_THREADS];
    __shared__ T vp[R], vd[YW_SEG];
    const YwItem it = items[blockIdx.x];
    const InstDesc& d = descs[it.inst];
    const int nt = d.n_tau, ny = d.n_y, tid = threadIdx.x;
    const int k = it.k0 + tid, j0 = it.j0;
    const bool act = k < nt;
    const double* vt = d.vel_tab + (size_t)node * 3 * ny;
    if (tid < R) vp[tid] = (T)vt[ny + ((j0 - 3 + tid) & (ny - 1))];
    if (tid < YW_SEG) vd[tid] = (T)vt[2 * ny + ((j0 + tid) & (ny - 1))];
    const T* uc = u + d.off_u + (act ? k : 0);
    #pragma unroll
    for (int r = 0; r < R; ++r) us[r][tid] = uc[(size_t)((j0 - 3 + r) & (ny - 1)) * nt];
    const T ay = (T)d.vel_amax[node];
    if (blockIdx.x == 0 && tid == 0 && (double)ay * d.h > d.cfl_max * d.dy) atomicOr(status, ST_CFL);
    __syncthreads();
    if (!act) return;
    const T eps = (T)d.weno_eps, idy = (T)(1.0 / d.dy);
    auto gp = [&](int r) -> T { const T x = us[r][tid]; return (T)0.5 * (vp[r] * x + ay * x); };
    auto gm = [&](int r) -> T { const T x = us[r][tid]; return (T)0.5 * (vp[r] * x - ay * x); };
    // face j0 - 1/2 (rows j0-3 .. j0+2 = r 0..5)
    T Gm = weno_face(gp(0), gp(1), gp(2), gp(3), gp(4), eps) + weno_face(gm(5), gm(4), gm(3), gm(2), gm(1), eps);
    T* bc = by + d.off_u + k;
    const int nj = min(YW_SEG, ny - j0);
    for (int i = 0; i < nj; ++i) {
        // face j0 + i + 1/2: rows r = i+1 .. i+6
        const T G = weno_face(gp(i + 1), gp(i + 2), gp(i + 3), gp(i + 4), gp(i + 5), eps) +
                    weno_face(gm(i + 6), gm(i + 5), gm(i + 4), gm(i + 3), gm(i + 2), eps);
        bc[(size_t)(j0 + i) * nt] = vd[i] * us[i + 3][tid] - (G - Gm) * idy;
        Gm = G;
    }
}

// Velocity tables (Sec. 2, Algorithm 1) of one instance at the nodes
// x_n = x0 + n h and rows y_j, evaluated in FP64 in Cartesian form:
// with K_n . r = (K_n lambda)(x cos theta_n + y sin theta_n) + phi_n and
// U~_n = a_n (-sin theta_n, cos theta_n),
//   U_par = sum -a_n sin theta_n cos(.),  U_perp = sum a_n cos theta_n cos(.),
//   d_y U_perp = -sum a_n cos theta_n (K_n lambda) sin theta_n sin(.).
// modes: [5][n_modes] = K_n lambda, a_n, cos theta_n, sin theta_n, phi_n.
// Block (j-range, node).
__global__ __launch_bounds__(256) void velocity_kernel(const InstDesc* __restrict__ descs, int inst,
                                                       const double* __restrict__ modes, int n_modes, double x0,
                                                       double h, double* __restrict__ tab) {
    const InstDesc& d = descs[inst];
    const int j = blockIdx.x * blockDim.x + threadIdx.x, n = blockIdx.y, ny = d.n_y;
    if (j >= ny) return;
    const double x = x0 + h * n, y = d.y0 + d.dy * j;
    const double* kl = modes;
    const double* am = modes + n_modes;
    const double* cth = modes + 2 * n_modes;
    const double* sth = modes + 3 * n_modes;
    const double* ph = modes + 4 * n_modes;
    double a = 0, p = 0, dp = 0;
    for (int m = 0; m < n_modes; ++m) {
        double sp, cp;
        sincos(kl[m] * (x * cth[m] + y * sth[m]) + ph[m], &sp, &cp);
        a -= am[m] * sth[m] * cp;
        p += am[m] * cth[m] * cp;
        dp -= am[m] * cth[m] * kl[m] * sth[m] * sp;
    }
    double* o = tab + (size_t)n * 3 * ny;
    o[j] = a;
    o[ny + j] = p;
    o[2 * ny + j] = dp;
}

// max_j |U_perp(x_n, y_j)| per node (one block per node)
__global__ __launch_bounds__(256) void velocity_max_kernel(const InstDesc* __restrict__ descs, int inst,
                                                           const double* __restrict__ tab,
                                                           double* __restrict__ amax) {
    __shared__ double red[4];
    const InstDesc& d = descs[inst];
    const int n = blockIdx.x, ny = d.n_y;
    const double* p = tab + (size_t)n * 3 * ny + ny;
    double m = 0;
    for (int j = threadIdx.x; j < ny; j += blockDim.x) m = fmax(m, fabs(p[j]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) amax[n] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ------------------------------------------------------------------ mean tau-mode (regularised multiplier)
// With the regularised multiplier the mean tau-mode of wavenumber ky has the
// real symbol l_0 = -(Dbar/2) ky^2 (4 pi / eps).  Column 0 of the spectral
// arrays holds the mean mode (.x) and the tau-Nyquist mode (.y) of every row
// in y-physical form; the y-pass leaves the mean as it is (the Nyquist part
// it updates pointwise).  This kernel applies the multipliers of l_0 along y:
//   after stage 1:  C~*(0, .) = F^-1[E_0 U^ + h Phi1_0 b^],
//                   P(0, .)   = F^-1[E_0 U^ + h (Phi1_0 - Phi2_0) b^],
//   after stage 2:  U(0, .) = C~(0, .) = P(0, .) + F^-1[h Phi2_0 b*^],
// U^ the y-transform of the state's mean column, b^ that of the mean of b.
// The flux difference of the Burgers and axial terms has no mean (sigma_0 =
// 0), so b^ comes from the transverse transport part only (By column 0) and
// is zero without transport (stage 2 then has nothing to do).  Two real
// columns share one complex transform each way: z = U + i b forward, and
// C~* + i P backward.  One block per instance; the FFT runs on the first
// n_y/16 threads.
template <typename T, int STAGE>
__global__ __launch_bounds__(512) void dc_kernel(const InstDesc* __restrict__ descs, cpx<T>* __restrict__ C,
                                                 cpx<T>* __restrict__ P, cpx<T>* __restrict__ U,
                                                 const cpx<T>* __restrict__ By, const cpx<T>* __restrict__ twst,
                                                 int step) {
    __shared__ alignas(32) cpx<T> lds[padded(8192)];
    const InstDesc& d = descs[blockIdx.x];
    if (!(d.reg_eps > 0.0)) return;
    const bool tb = d.vel != 0 && By != nullptr;
    if (STAGE == 2 && !tb) return;
    const int Ny = d.n_y, W = d.W, tid = threadIdx.x;
    const long long o = d.off_state;             // tile 0: element (y, column 0) at y W
    for (int y = tid; y < Ny; y += blockDim.x) {
        const long long e = o + (long long)y * W;
        const T b = tb ? By[e].x : (T)0;
        lds[padi(y)] = STAGE == 1 ? cpx<T>{U[e].x, b} : cpx<T>{b, (T)0};
    }
    __syncthreads();
    const bool act = tid < (Ny >> 4);
    lds_fft<T, -1>(lds, 0, Ny, tid, act, twst);
    __syncthreads();
    const double Dbar = d.D_step ? d.D_step[step] : d.D_const;
    const double dl = d.reg_eps / (4.0 * KZK_PI);
    const double s = 1.0 / (double)Ny;           // of the inverse transform
    // pairs (n, Ny - n): Z_n = A_n + i B_n with A, B the spectra of the two real columns
    for (int n = tid; n <= (Ny >> 1); n += blockDim.x) {
        const int nm = (Ny - n) & (Ny - 1);
        const double ky = 2.0 * KZK_PI * (double)n / d.L_y;
        cpx<double> e, p1, p2;
        phis_f64(-d.h * 0.5 * Dbar * ky * ky / dl, 0.0, e, p1, p2);
        const T E0 = (T)(e.x * s), H1 = (T)(d.h * p1.x * s), H2 = (T)(d.h * p2.x * s);
        const cpx<T> zn = lds[padi(n)], zm = lds[padi(nm)];
        // A_n = (Z_n + conj Z_{-n})/2, B_n = (Z_n - conj Z_{-n})/(2i), and the same at -n
        const cpx<T> An = {(T)0.5 * (zn.x + zm.x), (T)0.5 * (zn.y - zm.y)};
        const cpx<T> Bn = {(T)0.5 * (zn.y + zm.y), (T)0.5 * (zm.x - zn.x)};
        const cpx<T> Am = conj(An), Bm = conj(Bn);
        cpx<T> wn, wm;
        if (STAGE == 1) {
            // W = (E_0 A + H1 B) + i (E_0 A + (H1 - H2) B)
            const cpx<T> u1 = E0 * An + H1 * Bn, q1 = E0 * An + (H1 - H2) * Bn;
            const cpx<T> u2 = E0 * Am + H1 * Bm, q2 = E0 * Am + (H1 - H2) * Bm;
            wn = u1 + mul_si<1>(q1);
            wm = u2 + mul_si<1>(q2);
        } else {
            // W = H2 A (the transform of b* sits in A)
            wn = H2 * An;
            wm = H2 * Am;
        }
        lds[padi(n)] = wn;
        if (nm != n) lds[padi(nm)] = wm;
    }
    __syncthreads();
    lds_fft<T, 1>(lds, 0, Ny, tid, act, twst);
    __syncthreads();
    for (int y = tid; y < Ny; y += blockDim.x) {
        const long long e = o + (long long)y * W;
        const cpx<T> w = lds[padi(y)];
        if (STAGE == 1) {
            C[e].x = w.x;
            P[e].x = w.y;
        } else {
            const T v = P[e].x + w.x;
            C[e].x = v;
            U[e].x = v;
        }
    }
}

// ------------------------------------------------------------------ y-pass
// Tile <-> LDS copies.  Element e = j * W + c of a tile (global order) sits
// in LDS column c at logical c * n_y + j.  A thread moves the elements
// e = tid + q * NT (q < 16; a tile holds at most 16 NT elements) and issues
// all of its global loads before the first one is used.
__device__ __forceinline__ int tile_li(int e, int W, int lw, int Ny) { return padi((e & (W - 1)) * Ny + (e >> lw)); }

template <typename T, int NT>
__device__ __forceinline__ void tile_load(cpx<T>* lds, const cpx<T>* __restrict__ g, int ne, int tid, int W, int lw,
                                          int Ny, cpx<T> (&v)[16]) {
    // out-of-range slots reload the last element (no branch around the loads)
    #pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = g[min(tid + q * NT, ne - 1)];
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + q * NT;
        if (e < ne) lds[tile_li(e, W, lw, Ny)] = v[q];
    }
}

// The same in two steps, the loads into registers (real and imaginary parts
// in separate arrays, which the compiler keeps in registers also in FP64
// inside the persistent loop) and their LDS writes.
template <typename T, int NT>
__device__ __forceinline__ void tile_fetch(const cpx<T>* __restrict__ g, int ne, int tid, T (&vr)[16],
                                           T (&vi)[16]) {
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const cpx<T> x = g[min(tid + q * NT, ne - 1)];
        vr[q] = x.x;
        vi[q] = x.y;
    }
}

template <typename T, int NT>
__device__ __forceinline__ void tile_put(cpx<T>* lds, const T (&vr)[16], const T (&vi)[16], int ne, int tid, int W,
                                         int lw, int Ny) {
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + q * NT;
        if (e < ne) lds[tile_li(e, W, lw, Ny)] = cpx<T>{vr[q], vi[q]};
    }
}

// skips column 0 of the first tile (col0), whose modes are handled pointwise
template <typename T, int NT, bool NTS = false>
__device__ __forceinline__ void tile_store(cpx<T>* __restrict__ g, const cpx<T>* lds, int ne, int tid, int W, int lw,
                                           int Ny, bool col0) {
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + q * NT;
        if (e < ne && !(col0 && (e & (W - 1)) == 0)) {
            if constexpr (NTS) st_nt(g + e, lds[tile_li(e, W, lw, Ny)]);
            else g[e] = lds[tile_li(e, W, lw, Ny)];
        }
    }
}

// A block owns W adjacent tau-mode columns m0..m0+W-1 over all n_y rows.
// The mixed spectra C~, B~ (tau-spectral, y-physical) are stored in column
// tiles [m / W][y][m % W], so the tile is one contiguous block of W * n_y
// values; in LDS each column is contiguous (logical c * n_y + y) and n_y/16
// threads run its y-FFT.  The fully spectral state U and the stage value P
// are stored tile-contiguously at [m0 * n_y + e] in the same element order
// (e = y-wavenumber index * W + c).  The multiplier tables are stored per
// tile as tab[m0 * Nh + n * W + c] (n = |ky index|, the symbol is even in
// ky), pre-scaled by 1/n_y for the inverse y-transform.
//
// STAGE 0: U = F_y C~                           (start of a march)
// STAGE 1: U* = E U + h Phi1 F_y B~,  P = E U + h (Phi1 - Phi2) F_y B~,
//          C~* = F_y^-1 U*
// STAGE 2: U^{n+1} = P + h Phi2 F_y B~*,  C~^{n+1} = F_y^-1 U^{n+1}
// (F_y unnormalised; U is kept unnormalised, P and the inputs of the inverse
// transform carry the factor 1/n_y of the pre-scaled tables.)
// Column 0 holds the DC (.x) and tau-Nyquist (.y) modes in y-physical form in
// every array; its DC is invariant and its Nyquist multipliers are scalars.
// FP32 blocks of up to 512 threads are held to 128 VGPRs so that several
// share a compute unit (as many as their LDS allows).
//
// FULL (every instance has W n_y = 16 NT and n_y >= 512): element
// e = tid + q NT of a tile is row j0 + q dq of column c (c = tid mod W,
// j0 = tid / W, dq = n_y/16, a multiple of 32), so its global offset moves by
// the uniform q NT (buffer accesses with a per-thread base) and its padded
// LDS slot by the uniform q (dq + dq/16); no slot is out of range, and the
// first column of the first tile is one per-thread predicate.  Columns start
// at LDS slot c (P + 32) + (c R mod 32) (P = padded n_y, a multiple of 32
// slots apart, so every column would start on bank 0; R = 32/W rows of a
// column per half-wave): the LDS serves a 64-bit access of 32 lanes per
// cycle from 64 four-byte banks, and in the tile copies and the combine the
// W row runs of one half-wave (R rows of 8 bytes each) then cover the banks
// once instead of W/2 times (2-way conflicts at W = 4 with R = 64/W).
//
// Cache policy: every store of stages 1 and 2 (P, U, C~, the h Phi2 table)
// is non-temporal: each is read back only by a later kernel, after other
// arrays have streamed through, so keeping the written lines in L2 and the
// Infinity Cache mostly evicts lines the blocks are still reading.  NTL (full
// tiles with an FP64 state whose arrays outgrow the caches): the loads of U,
// P and the tables, read once per step, are non-temporal as well.  In FP32,
// and on arrays the 256 MB Infinity Cache holds, cached loads measured faster.
//
// S: precision of the spectral state U and the stage value P (T, or double
// in FP32 plans that keep their state in FP64: the combine then runs in FP64
// with the step's multipliers evaluated in FP64, and only the inputs of the
// inverse y-transform are rounded to T).
//
// LTW: the twiddles of every column transform are loaded per transform
// stage (with look-ahead) instead of held in registers across tiles.  Taken
// by full tiles when some instance has n_y = 8192 (whose transform has three
// stages with twiddles, more than the registers hold beside the tile), and
// by the FP32 general-tile blocks, whose element indexing leaves no room for
// held twiddles under the 128-VGPR cap (they would spill about 120 VGPRs to
// scratch; the loaded form spills 2 and gives bit-identical results).
template <typename T, int NT, int STAGE, bool FULL, typename S = T, bool LTW = false, bool NTL = false>
__global__ __launch_bounds__(NT, (sizeof(T) == 4 && NT <= 512) ? 4 : 1) void y_kernel(
        const InstDesc* __restrict__ descs, const YItem* __restrict__ items, int n_items, cpx<T>* __restrict__ C,
        const cpx<T>* __restrict__ B, const cpx<T>* __restrict__ By, cpx<S>* __restrict__ P, cpx<S>* __restrict__ U,
        cpx<T>* __restrict__ tabs, const cpx<T>* __restrict__ twst, int step) {
    __shared__ alignas(32) cpx<T> lds[padded(NT * 16) + (FULL ? NT : 0)];
    constexpr unsigned E = sizeof(cpx<T>);
    // byte offsets of tile elements in the state arrays are ES times those in the others
    constexpr unsigned ES = sizeof(cpx<S>) / sizeof(cpx<T>);
    constexpr bool S64 = !std::is_same<S, T>::value;
    // full tiles: loads of U, P and the tables (NTL)
    constexpr int CPL = NTL ? CP_NT : 0;
    const int tid = threadIdx.x;
    // Persistent blocks: block b takes the tiles b, b + gridDim.x, ...
    const cpx<T>* src = STAGE == 0 ? C : B;
    T vr[16], vi[16];
    // Stockham twiddles of this thread's column transform, loaded once per
    // transform length and held in registers for every tile (forward and
    // inverse), so no tile waits on twiddle loads.
    cpx<T> ytw[2][15];
    int tw_ny = 0;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const YItem it = items[item];
    const InstDesc& d = descs[it.inst];
    const int Ny = d.n_y, W = d.W, lw = d.log2W, Nh = d.Nh;
    const int m0 = it.m0;
    const int lt = ilog2(Ny) - 4;                 // log2 of the FFT threads per column
    const bool act = tid < (W << lt);
    const int fc = tid >> lt, ft = tid & ((1 << lt) - 1);
    const int ne = W * Ny;
    const long long to = d.off_state + (long long)m0 * Ny;
    const cpx<T>* Bt = B + to;
    cpx<T>* Ct = C + to;
    cpx<S>* Pt = P + to;
    cpx<S>* Ut = U + to;
    const cpx<T>* tE = tabs + d.off_tab + (long long)m0 * Nh;
    const cpx<T>* tP1 = tE + d.tab_stride;
    cpx<T>* tP2 = tabs + d.off_tab + (long long)m0 * Nh + 2 * d.tab_stride;
    const bool col0 = (m0 == 0);
    // tile element e = j * W + c (global order) <-> LDS column c at logical c * Ny + j
#define KZK_LI(e) padi((((e) & (W - 1)) * Ny) + ((e) >> lw))
    // x-dependent D: stage 1 computes the multipliers of this step (FP64)
    // instead of reading tables rebuilt every step, and stores h Phi2 / n_y
    // into its table for stage 2
    // (always, with an FP64 state: the stored tables are in T)
    const bool otf = STAGE == 1 && (S64 || d.D_step != nullptr);
    // FULL geometry (unused otherwise)
    const int c = tid & (W - 1), j0 = tid >> lw;
    const int dq = Ny >> 4, sq = dq + (dq >> 4);
    const int Pn = Ny + (Ny >> 4);
    // (full tiles have W <= 32; the general path does not use these slots)
    auto colbase = [&](int col) { return col * (Pn + 32) + (lw <= 5 ? ((col << (5 - lw)) & 31) : 0); };
    const int s0 = colbase(c) + padi(j0);               // slot of row j0 (q = 0)
    const int s1 = colbase(c) + padi(Ny - j0);          // slot of row Ny - j0 (q = 0)
    const bool keep_c = !(col0 && c == 0);
    // the tau-pass leaves the spectrum of the face fluxes; b^ = sigma F^ (the
    // column of a thread's combine items is tid mod W in both paths).  With
    // transport the transverse part By (a spectrum of b itself) is added at
    // the tile load, sigma F^ + By, and the combine multiplies by 1.
    const bool tr = STAGE > 0 && By != nullptr && d.vel != 0;
    const cpx<T> sgl = STAGE > 0 ? flux_diff_symbol<T>(d, m0 + c) : cpx<T>{(T)0, (T)0};
    const cpx<T> sg = tr ? cpx<T>{(T)1, (T)0} : sgl;
    cpx<T>* fbuf = FULL ? lds + colbase(fc) : lds;      // this thread's FFT column
    const int fbase = FULL ? 0 : fc * Ny;

    if constexpr (FULL) {
        const auto rs = buf_rsrc(src + to);
        #pragma unroll
        for (int q = 0; q < 16; ++q) {
            const cpx<T> x = buf_ld<T>(rs, tid * E, q * NT * E);
            vr[q] = x.x;
            vi[q] = x.y;
        }
    } else {
        tile_fetch<T, NT>(src + to, ne, tid, vr, vi);
    }
    if (tr) {
        #pragma unroll
        for (int q = 0; q < 16; ++q) {
            const cpx<T> y = By[to + min(tid + q * NT, ne - 1)];
            const cpx<T> x = cmul(sgl, cpx<T>{vr[q], vi[q]}) + y;
            vr[q] = x.x;
            vi[q] = x.y;
        }
    }
    if (Ny != tw_ny) {
        if constexpr (!LTW) lds_fft_twiddles<T>(Ny, ft, twst, ytw);
        tw_ny = Ny;
    }
    if constexpr (FULL) {
        #pragma unroll
        for (int q = 0; q < 16; ++q) lds[s0 + q * sq] = cpx<T>{vr[q], vi[q]};
    } else {
        tile_put<T, NT>(lds, vr, vi, ne, tid, W, lw, Ny);
    }
    __syncthreads();
    if (STAGE == 0) {
        if constexpr (LTW) lds_fft<T, -1>(fbuf, fbase, Ny, ft, act, twst);
        else lds_fft_held<T, -1>(fbuf, fbase, Ny, ft, act, ytw);
        if constexpr (FULL) {
            const auto rc = buf_rsrc(Ct), ru = buf_rsrc(Ut);
            #pragma unroll
            for (int q = 0; q < 16; ++q)
                buf_st<S>(ru, ES * tid * E, ES * q * NT * E,
                          cvs<S>(keep_c ? lds[s0 + q * sq] : buf_ld<T>(rc, tid * E, q * NT * E)));
        } else {
            #pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = tid + q * NT;
                if (e < ne) Ut[e] = cvs<S>((col0 && (e & (W - 1)) == 0) ? Ct[e] : lds[KZK_LI(e)]);
            }
        }
        __syncthreads();
        continue;
    }

    if constexpr (LTW) lds_fft<T, -1>(fbuf, fbase, Ny, ft, act, twst);
    else lds_fft_held<T, -1>(fbuf, fbase, Ny, ft, act, ytw);
    // combine: the symbol is even in ky, so one table row n serves y-wavenumber
    // indices n and Ny - n.  A thread has at most 9 half-tile items
    // (Nh * W <= 8 NT + W); their global loads are issued before use.
    const int nh = Nh * W;
    constexpr int QH = 9;
    if constexpr (FULL) {
        // item q: h = tid + q NT, row n = j0 + q dq; q < 8 for every thread,
        // q = 8 (n = Ny/2) for tid < W only.  The partner row Ny - n exists
        // for q = 1..7 and for q = 0 with j0 > 0; its element is
        // ne - tid + 2c - q NT.
        const auto rU = buf_rsrc(Ut), rP = buf_rsrc(Pt), rE = buf_rsrc(tE), rP1 = buf_rsrc(tP1), rP2 = buf_rsrc(tP2);
        const bool first = tid < W;                    // rows 0 and Ny/2 of column c
        const unsigned v0 = tid * E;                   // element h at q = 0
        const unsigned v8 = min(tid, W - 1) * E;       // h at q = 8, clamped to the tile's table rows
        const unsigned vm = (unsigned)(ne - tid + 2 * c - 8 * NT) * E;   // partner at q = 8 (base)
        const unsigned vm0 = first ? v0 : (unsigned)(ne - tid + 2 * c) * E;  // partner at q = 0
        auto vpart = [&](int q) { return q == 0 ? vm0 : vm; };
        auto spart = [&](int q) { return q == 0 ? 0u : (unsigned)(8 - q) * NT * E; };
        auto vself = [&](int q) { return q == 8 ? v8 : v0; };
        if (STAGE == 1 && otf) {
            // one item at a time (the FP64 multiplier code needs the registers);
            // the U loads of the next item are in flight during this item's
            // multipliers.  Column 0 of the first tile is handled pointwise below.
            cpx<S> u0 = buf_ld<S, CPL>(rU, ES * v0, 0), u1 = buf_ld<S, CPL>(rU, ES * vm0, 0);
            #pragma unroll
            for (int q = 0; q < QH; ++q) {
                cpx<S> x0 = u0, x1 = u1;
                if (q + 1 < QH) {
                    x0 = buf_ld<S, CPL>(rU, ES * vself(q + 1), ES * (q + 1) * NT * E);
                    if (q + 1 < 8) x1 = buf_ld<S, CPL>(rU, ES * vpart(q + 1), ES * spart(q + 1));
                }
                if (q < 8 || first) {
                    const int n = j0 + q * dq;
                    const bool two = q > 0 ? q < 8 : !first;
                    cpx<S> E0 = {(S)0, (S)0}, P1 = E0, P2 = E0;
                    if (m0 + c > 0) {
                        mode_multipliers<S>(d, m0 + c, n, step, E0, P1, P2);
                    } else if (n == 0) {
                        S e, p1, p2;
                        nyquist_multipliers<S>(d, e, p1, p2);
                        P2 = cpx<S>{p2, (S)0};
                    }
                    buf_st<T, CP_NT>(rP2, vself(q), q * NT * E, cvs<T>(P2));
                    {
                        const int li = s0 + q * sq;
                        const cpx<S> bh = cvs<S>(cmul(sg, lds[li]));
                        const cpx<S> EU = cmul(E0, u0);
                        if (keep_c) buf_st<S, CP_NT>(rP, ES * vself(q), ES * q * NT * E, EU + cmul(P1 - P2, bh));
                        lds[li] = cvs<T>(EU + cmul(P1, bh));
                    }
                    if (two) {
                        const int li = s1 - q * sq;
                        const cpx<S> bh = cvs<S>(cmul(sg, lds[li]));
                        const cpx<S> EU = cmul(E0, u1);
                        if (keep_c) buf_st<S, CP_NT>(rP, ES * vpart(q), ES * spart(q), EU + cmul(P1 - P2, bh));
                        lds[li] = cvs<T>(EU + cmul(P1, bh));
                    }
                }
                u0 = x0;
                u1 = x1;
            }
        } else {
            // the loads of three items are issued before use (nine at once
            // need more registers than the held twiddles leave; reloading the
            // twiddles per transform to make room measured much slower)
            constexpr int QB = 3;
            #pragma unroll
            for (int q0 = 0; q0 < QH; q0 += QB) {
                cpx<T> tb[QB][3];
                cpx<S> ua[QB][2];
                #pragma unroll
                for (int q = 0; q < QB; ++q) {
                    const int qq = q0 + q;
                    const unsigned vs = vself(qq), ss = qq * NT * E;
                    if (STAGE == 1) {
                        tb[q][0] = buf_ld<T, CPL>(rE, vs, ss);
                        tb[q][1] = buf_ld<T, CPL>(rP1, vs, ss);
                        tb[q][2] = buf_ld<T, CPL>(rP2, vs, ss);
                        ua[q][0] = buf_ld<S, CPL>(rU, ES * vs, ES * ss);
                        ua[q][1] = qq < 8 ? buf_ld<S, CPL>(rU, ES * vpart(qq), ES * spart(qq)) : ua[q][0];
                    } else {
                        tb[q][2] = buf_ld<T, CPL>(rP2, vs, ss);
                        ua[q][0] = buf_ld<S, CPL>(rP, ES * vs, ES * ss);
                        ua[q][1] = qq < 8 ? buf_ld<S, CPL>(rP, ES * vpart(qq), ES * spart(qq)) : ua[q][0];
                    }
                }
                #pragma unroll
                for (int q = 0; q < QB; ++q) {
                    const int qq = q0 + q;
                    if (!(qq < 8 || first)) continue;
                    const bool two = qq > 0 ? qq < 8 : !first;
                    #pragma unroll
                    for (int pass = 0; pass < 2; ++pass) {
                        if (pass == 1 && !two) break;
                        const int li = pass ? s1 - qq * sq : s0 + qq * sq;
                        const unsigned vv = pass ? vpart(qq) : vself(qq);
                        const unsigned ss = pass ? spart(qq) : (unsigned)qq * NT * E;
                        const cpx<S> bh = cvs<S>(cmul(sg, lds[li]));
                        if (STAGE == 1) {
                            const cpx<S> EU = cmul(cvs<S>(tb[q][0]), ua[q][pass]);
                            if (keep_c) buf_st<S, CP_NT>(rP, ES * vv, ES * ss, EU + cmul(cvs<S>(tb[q][1] - tb[q][2]), bh));
                            lds[li] = cvs<T>(EU + cmul(cvs<S>(tb[q][1]), bh));
                        } else {
                            const cpx<S> un = ua[q][pass] + cmul(cvs<S>(tb[q][2]), bh);
                            if (keep_c) buf_st<S, CP_NT>(rU, ES * vv, ES * ss, (S)Ny * un);
                            lds[li] = cvs<T>(un);
                        }
                    }
                }
            }
        }
    } else if (STAGE == 1 && otf) {
        // one item at a time (the FP64 multiplier code needs the registers);
        // the U loads of the next item are in flight during this item's
        // multipliers.  Column 0 of the first tile is handled pointwise below
        // (its combine values are never stored); its table slots hold the
        // tau-Nyquist scalars (n = 0) and zeros, as the tables kernel's.
        cpx<S> u0, u1;
        {
            const int h = min(tid, nh - 1);
            const int n = h >> lw, cc = h & (W - 1);
            const int j2 = (n == 0 || 2 * n == Ny) ? n : Ny - n;
            u0 = Ut[n * W + cc];
            u1 = Ut[j2 * W + cc];
        }
        #pragma unroll
        for (int q = 0; q < QH; ++q) {
            cpx<S> x0 = u0, x1 = u1;
            if (q + 1 < QH) {
                const int hn = min(tid + (q + 1) * NT, nh - 1);
                const int n = hn >> lw, cc = hn & (W - 1);
                const int j2 = (n == 0 || 2 * n == Ny) ? n : Ny - n;
                x0 = Ut[n * W + cc];
                x1 = Ut[j2 * W + cc];
            }
            const int h = tid + q * NT;
            if (h < nh) {
                const int n = h >> lw, cc = h & (W - 1);
                const bool keep_col = !(col0 && cc == 0);
                const bool two = !(n == 0 || 2 * n == Ny);
                cpx<S> E = {(S)0, (S)0}, P1 = E, P2 = E;
                if (m0 + cc > 0) {
                    mode_multipliers<S>(d, m0 + cc, n, step, E, P1, P2);
                } else if (n == 0) {
                    S e, p1, p2;
                    nyquist_multipliers<S>(d, e, p1, p2);
                    P2 = cpx<S>{p2, (S)0};
                }
                st_nt(tP2 + h, cvs<T>(P2));
                #pragma unroll
                for (int pass = 0; pass < 2; ++pass) {
                    if (pass == 1 && !two) break;
                    const int j = pass ? Ny - n : n;
                    const int e = j * W + cc, li = padi(cc * Ny + j);
                    const cpx<S> bh = cvs<S>(cmul(sg, lds[li]));
                    const cpx<S> EU = cmul(E, pass ? u1 : u0);
                    if (keep_col) st_nt(Pt + e, EU + cmul(P1 - P2, bh));
                    lds[li] = cvs<T>(EU + cmul(P1, bh));
                }
            }
            u0 = x0;
            u1 = x1;
        }
    } else {
    #pragma unroll
    for (int q0 = 0; q0 < QH; q0 += 3) {
        cpx<T> tb[3][3];
        cpx<S> ua[3][2];
        #pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int h = min(tid + (q0 + q) * NT, nh - 1);   // clamped: loads without a branch
            const int n = h >> lw, cc = h & (W - 1);
            const int j2 = (n == 0 || 2 * n == Ny) ? n : Ny - n;
            if (STAGE == 1) {
                tb[q][0] = tE[h];
                tb[q][1] = tP1[h];
                tb[q][2] = tP2[h];
                ua[q][0] = Ut[n * W + cc];
                ua[q][1] = Ut[j2 * W + cc];
            } else {
                tb[q][2] = tP2[h];
                ua[q][0] = Pt[n * W + cc];
                ua[q][1] = Pt[j2 * W + cc];
            }
        }

        #pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int h = tid + (q0 + q) * NT;
            if (!(q0 + q < QH && h < nh)) continue;
            const int n = h >> lw, cc = h & (W - 1);
            const bool keep_col = !(col0 && cc == 0);
            const bool two = !(n == 0 || 2 * n == Ny);
            #pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                if (pass == 1 && !two) break;
                const int j = pass ? Ny - n : n;
                const int e = j * W + cc, li = padi(cc * Ny + j);
                const cpx<S> bh = cvs<S>(cmul(sg, lds[li]));
                if (STAGE == 1) {
                    const cpx<S> EU = cmul(cvs<S>(tb[q][0]), ua[q][pass]);
                    if (keep_col) st_nt(Pt + e, EU + cmul(cvs<S>(tb[q][1] - tb[q][2]), bh));
                    lds[li] = cvs<T>(EU + cmul(cvs<S>(tb[q][1]), bh));
                } else {
                    // un = U^{n+1} / n_y (the tables carry the 1/n_y of the inverse y-FFT);
                    // the state keeps the unnormalised spectrum (a power-of-two scaling, exact)
                    const cpx<S> un = ua[q][pass] + cmul(cvs<S>(tb[q][2]), bh);
                    if (keep_col) st_nt(Ut + e, (S)Ny * un);
                    lds[li] = cvs<T>(un);
                }
            }
        }
    }
    }
    __syncthreads();
    if constexpr (LTW) lds_fft<T, 1>(fbuf, fbase, Ny, ft, act, twst);
    else lds_fft_held<T, 1>(fbuf, fbase, Ny, ft, act, ytw);
    if constexpr (FULL) {
        const auto rc = buf_rsrc(Ct);
        // an opaque copy of the base slot, so that the compiler recomputes the
        // 16 slots here instead of keeping those of the tile load live in
        // registers through both transforms and the combine
        int sb = s0;
        asm volatile("" : "+v"(sb));
        if (keep_c) {
            #pragma unroll
            for (int q = 0; q < 16; ++q) buf_st<T, CP_NT>(rc, tid * E, q * NT * E, lds[sb + q * sq]);
        }
    } else {
        tile_store<T, NT, true>(Ct, lds, ne, tid, W, lw, Ny, col0);
    }
#undef KZK_LI
    if (col0) {
        // DC (.x) is invariant; the tau-Nyquist (.y) multipliers are ky-independent scalars
        S EN, P1N, P2N;
        if (otf) {
            nyquist_multipliers<S>(d, EN, P1N, P2N);
        } else {
            EN = tE[0].x;
            P1N = tP1[0].x;
            P2N = tP2[0].x;
        }
        const T sN = (T)(-2.0 / d.dtau);                  // sigma at the tau-Nyquist mode
        for (int y = tid; y < Ny; y += NT) {
            const long long o = (long long)y * W;
            // the mean mode (.x) is left to the DC path: zeroed F(b)(0, .), or
            // the mean-column kernel of the regularised multiplier
            const S by = (S)(sN * Bt[o].y + (tr ? By[to + o].y : (T)0));
            if (STAGE == 1) {
                const cpx<S> cr = Ut[o];
                Ct[o] = cvs<T>(cpx<S>{cr.x, EN * cr.y + P1N * by});
                Pt[o] = cpx<S>{cr.x, EN * cr.y + (P1N - P2N) * by};
            } else {
                const cpx<S> p = Pt[o];
                const cpx<S> un = cpx<S>{p.x, p.y + P2N * by};
                Ct[o] = cvs<T>(un);
                Ut[o] = un;
            }
        }
    }
    __syncthreads();    // LDS reads of this tile are done before the next tile is written
    }
}

// ------------------------------------------------------------------ adjoint
// Transpose of the step map u^n -> u^{n+1} (ExpRK22, Sec. 3.3 eq. (19)) on
// real fields.  With Ecal = F^-1 E F, Pk = F^-1 Phi_k Z F (Z zeroes the mean
// tau-mode) and J0, J1 the Jacobians of b at (x_n, u^n) and (x_{n+1}, u*):
//     mu    = h J1^T P2^T lam
//     lam_n = Ecal^T (lam + mu) + h J0^T [ (P1 - P2)^T lam + P1^T mu ].
// The transpose of a Fourier multiplier is the multiplier with the complex
// conjugate symbol (the symbol is Hermitian), so the adjoint reuses the tables.

// Sum over the tpr threads of one line (same grouping as line_max).
template <typename T>
__device__ __forceinline__ T line_sum(T v, int tpr, T* red) {
    const int w = tpr < 64 ? tpr : 64;
    for (int o = w >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (tpr > 64) {
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = v;
        __syncthreads();
        const int nw = tpr >> 6, first = (threadIdx.x / tpr) * nw;
        T m = red[first];
        for (int i = 1; i < nw; ++i) m += red[first + i];
        v = m;
        __syncthreads();
    }
    return v;
}

// Gradient of weno_face with respect to v0..v4:
//   dF/dv_k = sum_r w_r dq_r/dv_k + sum_r c_r dbeta_r/dv_k,
//   c_r = -2 (q_r - F) w_r / (eps + beta_r),  w_r the nonlinear weights.
template <typename T>
__device__ __forceinline__ void weno_face_grad(T v0, T v1, T v2, T v3, T v4, T eps, T g[5]) {
    const T c1312 = (T)(13.0 / 12.0), c136 = (T)(13.0 / 6.0), s6 = (T)(1.0 / 6.0);
    T q0 = ((T)2 * v0 - (T)7 * v1 + (T)11 * v2) * s6;
    T q1 = (-v1 + (T)5 * v2 + (T)2 * v3) * s6;
    T q2 = ((T)2 * v2 + (T)5 * v3 - v4) * s6;
    T A0 = v0 - (T)2 * v1 + v2, B0 = v0 - (T)4 * v1 + (T)3 * v2;
    T A1 = v1 - (T)2 * v2 + v3, B1 = v1 - v3;
    T A2 = v2 - (T)2 * v3 + v4, B2 = (T)3 * v2 - (T)4 * v3 + v4;
    const T S0 = eps + c1312 * A0 * A0 + (T)0.25 * B0 * B0;
    const T S1 = eps + c1312 * A1 * A1 + (T)0.25 * B1 * B1;
    const T S2 = eps + c1312 * A2 * A2 + (T)0.25 * B2 * B2;
    // 1/S_r from one reciprocal of the product (S_r >= eps, so the product stays normal)
    const T s12 = S1 * S2, s02 = S0 * S2, s01 = S0 * S1, iP = rcp(S0 * s12);
    T r0 = s12 * iP, r1 = s02 * iP, r2 = s01 * iP;
    T a0 = (T)0.1 * r0 * r0, a1 = (T)0.6 * r1 * r1, a2 = (T)0.3 * r2 * r2;
    T iS = rcp(a0 + a1 + a2);
    T w0 = a0 * iS, w1 = a1 * iS, w2 = a2 * iS;
    T F = w0 * q0 + w1 * q1 + w2 * q2;
    T c0 = (T)-2 * (q0 - F) * w0 * r0;
    T c1 = (T)-2 * (q1 - F) * w1 * r1;
    T c2 = (T)-2 * (q2 - F) * w2 * r2;
    T e0 = c136 * A0 * c0, f0 = (T)0.5 * B0 * c0;
    T e1 = c136 * A1 * c1, f1 = (T)0.5 * B1 * c1;
    T e2 = c136 * A2 * c2, f2 = (T)0.5 * B2 * c2;
    g[0] = (T)2 * s6 * w0 + e0 + f0;
    g[1] = (T)-7 * s6 * w0 - s6 * w1 - (T)2 * e0 - (T)4 * f0 + e1 + f1;
    g[2] = (T)11 * s6 * w0 + (T)5 * s6 * w1 + (T)2 * s6 * w2 + e0 + (T)3 * f0 - (T)2 * e1 + e2 + (T)3 * f2;
    g[3] = (T)2 * s6 * w1 + (T)5 * s6 * w2 + e1 - f1 - (T)2 * e2 - (T)4 * f2;
    g[4] = -s6 * w2 + e2 + f2;
}

// Transpose of the WENO5/LF b on one line, including the dependence of the
// LF speed alpha = |nl| max|u| on u (its sub-gradient split over ties).
// ubuf: the line u (logical base ub); gbuf: the cotangent of b (base gb).
// Returns the result for the thread's own points 4c..4c+3 of its chunks
// c = t + q*tpr in out[q][.].  Both buffers are overwritten (halo exchange).
// GK > 0: M = 7 * 2^GK (chunk indices wrap by a select); tpg: threads of a
// line's group for the line sums (tpr for power-of-two M).
template <typename T, int GK = 0>
__device__ __forceinline__ void weno_adjoint_line(cpx<T>* lds, int ub, int gb, int M, int t, int tpr, int tpg,
                                                  bool active, T nlT, T mx, T eps, T dtau, T* redT, T out[8][4]) {
    const int Nc = M >> 1;
    auto wrapc = [&](int c) { return GK > 0 ? (c < 0 ? c + Nc : (c >= Nc ? c - Nc : c)) : (c & (Nc - 1)); };
    const T alpha = (T)fabs(nlT) * mx;
    const T idt = (T)1 / dtau;
    T halo[8][5];
    T abar = 0, nties = 0;
    unsigned tie = 0, neg = 0;
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int c = t + q * tpr;
        #pragma unroll
        for (int i = 0; i < 4; ++i) out[q][i] = 0;
        #pragma unroll
        for (int i = 0; i < 5; ++i) halo[q][i] = 0;
        if (active) {
            quad<T> a = lds_quad(lds, ub, wrapc(c - 1)), b = lds_quad(lds, ub, c),
                    e = lds_quad(lds, ub, wrapc(c + 1));
            T u[12] = {a.v[0], a.v[1], a.v[2], a.v[3], b.v[0], b.v[1], b.v[2], b.v[3],
                       e.v[0], e.v[1], e.v[2], e.v[3]};
            quad<T> g0 = lds_quad(lds, gb, c), g1 = lds_quad(lds, gb, wrapc(c + 1));
            T gg[5] = {g0.v[0], g0.v[1], g0.v[2], g0.v[3], g1.v[0]};
            T fp[12], fm[12], accP[12], accM[12];
            #pragma unroll
            for (int i = 0; i < 12; ++i) { accP[i] = 0; accM[i] = 0; }
            #pragma unroll
            for (int i = 2; i <= 10; ++i) {
                T f = (T)0.5 * nlT * u[i] * u[i];
                fp[i] = (T)0.5 * (f + alpha * u[i]);
                fm[i] = (T)0.5 * (f - alpha * u[i]);
            }
            #pragma unroll
            for (int f = 0; f < 4; ++f) {
                // face 4c+f+1/2: b_i has -F/dtau, b_{i+1} has +F/dtau
                const T G = (gg[f + 1] - gg[f]) * idt;
                T dp[5], dm[5];
                weno_face_grad(fp[f + 2], fp[f + 3], fp[f + 4], fp[f + 5], fp[f + 6], eps, dp);
                weno_face_grad(fm[f + 7], fm[f + 6], fm[f + 5], fm[f + 4], fm[f + 3], eps, dm);
                #pragma unroll
                for (int r = 0; r < 5; ++r) {
                    accP[f + 2 + r] += G * dp[r];
                    accM[f + 7 - r] += G * dm[r];
                }
            }
            T contrib[12];
            #pragma unroll
            for (int i = 2; i <= 10; ++i) {
                const T hu = (T)0.5 * u[i];
                contrib[i] = accP[i] * ((T)0.5 * nlT * u[i] + (T)0.5 * alpha) +
                             accM[i] * ((T)0.5 * nlT * u[i] - (T)0.5 * alpha);
                abar += hu * (accP[i] - accM[i]);
            }
            #pragma unroll
            for (int i = 0; i < 4; ++i) {
                out[q][i] = contrib[4 + i];
                const T au = (T)fabs(u[4 + i]);
                if (au == mx && mx > (T)0) {
                    tie |= 1u << (4 * q + i);
                    nties += (T)1;
                }
                if (u[4 + i] < (T)0) neg |= 1u << (4 * q + i);
            }
            halo[q][0] = contrib[2];
            halo[q][1] = contrib[3];
            halo[q][2] = contrib[8];
            halo[q][3] = contrib[9];
            halo[q][4] = contrib[10];
        }
    }
    abar = line_sum(abar, tpg, redT);
    nties = line_sum(nties, tpg, redT);
    __syncthreads();
    // halo exchange: left halo (points 4c-2, 4c-1) into the u buffer slots
    // of chunk c; right halo (points 4c+4..4c+6) into the g buffer.
    T* ur = reinterpret_cast<T*>(lds);
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int c = t + q * tpr;
        if (active) {
            lds_quad_st(lds, ub, c, quad<T>{{halo[q][0], halo[q][1], (T)0, (T)0}});
            lds_quad_st(lds, gb, c, quad<T>{{halo[q][2], halo[q][3], halo[q][4], (T)0}});
        }
    }
    (void)ur;
    __syncthreads();
    const T aterm = nties > (T)0 ? abar * (T)fabs(nlT) / nties : (T)0;
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int c = t + q * tpr;
        if (active) {
            quad<T> lh = lds_quad(lds, ub, wrapc(c + 1));   // chunk c+1's left halo: points 4c+2, 4c+3
            quad<T> rh = lds_quad(lds, gb, wrapc(c - 1));   // chunk c-1's right halo: points 4c..4c+2
            out[q][0] += rh.v[0];
            out[q][1] += rh.v[1];
            out[q][2] += rh.v[2] + lh.v[0];
            out[q][3] += lh.v[1];
            #pragma unroll
            for (int i = 0; i < 4; ++i)
                if (tie & (1u << (4 * q + i))) out[q][i] += (neg & (1u << (4 * q + i))) ? -aterm : aterm;
        }
    }
    __syncthreads();
}

// Adjoint tau-pass.  STAGE 1: cotangent T~1 (mixed spectrum) and u* ->
// mu = J1^T t1 -> M~.  STAGE 2: T~2, R~ and u^n -> lam_n = r + J0^T t2 -> L~.
// (The factor h is carried by the pre-scaled tables of the adjoint y-pass.)
// GK > 0: every instance has M = 7 * 2^GK (lines in groups of 2^(GK-1)
// threads, as in the forward tau-kernel; tw is the table e^{-2 pi i k/n_tau}).
template <typename T, int STAGE, int GK = 0>
__global__ __launch_bounds__(TAU_THREADS) void tau_adj_kernel(const InstDesc* __restrict__ descs,
                                                              const TauItem* __restrict__ items,
                                                              const cpx<T>* __restrict__ Tin,
                                                              const cpx<T>* __restrict__ Rin,
                                                              const T* __restrict__ ustore,
                                                              cpx<T>* __restrict__ out,
                                                              const cpx<T>* __restrict__ tw,
                                                              const cpx<T>* __restrict__ twst, int log2_ntw, int node,
                                                              unsigned* __restrict__ status) {
    __shared__ alignas(32) cpx<T> lds[2 * padded(TAU_THREADS * 16)];
    __shared__ T redT[TAU_THREADS / 64];
    __shared__ int redI[TAU_THREADS / 64];
    const TauItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const InstDesc& d = descs[it.inst];
    constexpr int MG = GK > 0 ? (7 << GK) : 16;    // compile-time M of the 7 * 2^K lines
    const int M = GK > 0 ? MG : d.M, N = 2 * M;
    const int tpr = M >> 4;
    const int tpg = GK > 0 ? (1 << (GK - 1)) : tpr;
    const int r = threadIdx.x / tpg, t = threadIdx.x & (tpg - 1);
    const int row = it.row0 + r;
    const int rows = GK > 0 ? (TAU_THREADS >> (GK - 1)) : (TAU_THREADS * 16) / M;
    const bool active = (GK == 0 || t < tpr) && (r < rows) && (row < d.n_y);
    const int gb = r * M;                          // cotangent line
    const int ub = TAU_THREADS * 16 + r * M;        // u line (second half of the buffer)
    const SpecIdx ix = spec_idx(d.log2W, d.n_y, true);
    const long long so = d.off_state + ((long long)row << d.log2W);

    if (active) {
        if constexpr (GK > 0) c2r_pre_gen<T, MG>(Tin + so, ix, lds, gb, t, tw, (T)1 / (T)N);
        else c2r_pre(Tin + so, ix, lds, gb, M, t, tpr, tw, log2_ntw, (T)1 / (T)N);
    }
    // the stored physical line
    T mx = 0;
    int bad = 0;
    if (active) {
        const quad<T>* ug = reinterpret_cast<const quad<T>*>(ustore + d.off_u + (long long)row * N);
        quad<T> v[8];
        #pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = ug[t + q * tpr];
        #pragma unroll
        for (int q = 0; q < 8; ++q) {
            #pragma unroll
            for (int i = 0; i < 4; ++i) {
                bad |= !finite_val(v[q].v[i]);
                mx = tmax(mx, (T)fabs(v[q].v[i]));
            }
            lds_quad_st(lds, ub, t + q * tpr, v[q]);
        }
    }
    __syncthreads();
    if constexpr (GK > 0) gen_fft<T, 1, GK>(lds, gb, t, active, tw);
    else lds_fft<T, 1>(lds, gb, M, t, active, twst);
    mx = line_max(mx, tpg, redT);
    bad = line_or(bad, tpg, redI);
    if (active && t == 0 && bad) atomicOr(status, ST_NONFINITE);
    const double nl = d.nl_node ? d.nl_node[node] : d.nl_const;
    T res[8][4];
    weno_adjoint_line<T, GK>(lds, ub, gb, M, t, tpr, tpg, active, (T)nl, mx, (T)d.weno_eps, (T)d.dtau, redT, res);
    #pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int c = t + q * tpr;
        if (active) lds_quad_st(lds, gb, c, quad<T>{{res[q][0], res[q][1], res[q][2], res[q][3]}});
    }
    __syncthreads();
    if constexpr (GK > 0) gen_fft<T, -1, GK>(lds, gb, t, active, tw);
    else lds_fft<T, -1>(lds, gb, M, t, active, twst);
    // stage 2: lam_n = F_tau(J0^T t2) + R~ (the spectrum R~ is added after the
    // forward transform instead of transforming it back and forth)
    if (active) {
        if constexpr (GK > 0) r2c_post_gen<T, MG>(lds, gb, out + so, ix, t, tw, STAGE == 2 ? Rin + so : nullptr);
        else r2c_post(lds, gb, out + so, ix, M, t, tpr, tw, log2_ntw, STAGE == 2 ? Rin + so : nullptr);
    }
}

// Adjoint y-pass.  STAGE 1: L~ -> Lh = F_y L~ (kept, tile-contiguous) and
// T~1 = F_y^-1 conj(h Phi2) Z Lh.  STAGE 2: M~ and Lh ->
// T~2 = F_y^-1 Z [conj(h(Phi1 - Phi2)) Lh + conj(h Phi1) Mh] and
// R~ = F_y^-1 conj(E) (Lh + Mh).  Column 0 (DC, tau-Nyquist) pointwise in y;
// its Lh slot holds the raw column.  LTW: some instance has n_y = 8192,
// whose per-thread twiddles do not fit in registers beside the held
// values; stage 1 then loads them per transform stage as stage 2 does.
template <typename T, int NT, int STAGE, bool LTW = false>
__global__ __launch_bounds__(NT, (sizeof(T) == 4 && NT <= 512) ? 4 : 1) void y_adj_kernel(const InstDesc* __restrict__ descs,
                                                   const YItem* __restrict__ items, const cpx<T>* __restrict__ In,
                                                   cpx<T>* __restrict__ Lh, cpx<T>* __restrict__ Tout,
                                                   cpx<T>* __restrict__ Rout, const cpx<T>* __restrict__ tabs,
                                                   const cpx<T>* __restrict__ twst) {
    __shared__ alignas(32) cpx<T> lds[padded(NT * 16)];
    const YItem it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const InstDesc& d = descs[it.inst];
    const int Ny = d.n_y, W = d.W, lw = d.log2W, Nh = d.Nh;
    const int m0 = it.m0;
    const int tid = threadIdx.x;
    const int lt = ilog2(Ny) - 4;
    const bool act = tid < (W << lt);
    const int fc = tid >> lt, ft = tid & ((1 << lt) - 1);
    const int ne = W * Ny;
    const long long to = d.off_state + (long long)m0 * Ny;
    const cpx<T>* It = In + to;
    cpx<T>* Lt = Lh + to;
    cpx<T>* Tt = Tout + to;
    const cpx<T>* tE = tabs + d.off_tab + (long long)m0 * Nh;
    const cpx<T>* tP1 = tE + d.tab_stride;
    const cpx<T>* tP2 = tE + 2 * d.tab_stride;
    const bool col0 = (m0 == 0);
    const int half = Ny >> 1;
#define KZK_LI(e) padi((((e) & (W - 1)) * Ny) + ((e) >> lw))

    // Stage 1 holds this thread's twiddles in registers for both of its
    // transforms; stage 2 keeps 16 values per thread across its second
    // transform and loads its twiddles per transform stage instead.
    cpx<T> ytw[2][15];
    if constexpr (STAGE == 1 && !LTW) lds_fft_twiddles<T>(Ny, ft, twst, ytw);
    cpx<T> keep[16];
    tile_load<T, NT>(lds, It, ne, tid, W, lw, Ny, keep);
    __syncthreads();
    if constexpr (STAGE == 1 && !LTW)
        lds_fft_held<T, -1>(lds, fc * Ny, Ny, ft, act, ytw);
    else
        lds_fft<T, -1, false>(lds, fc * Ny, Ny, ft, act, twst);
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + q * NT;
        if (e < ne) {
            const int j = e >> lw, cc = e & (W - 1);
            const int n = j <= half ? j : Ny - j;
            const int ti = n * W + cc;
            const int li = KZK_LI(e);
            cpx<T> X = lds[li];
            if (STAGE == 1) {
                if (!(col0 && cc == 0)) Lt[e] = X;
                lds[li] = cmulc(X, tP2[ti]);
            } else {
                cpx<T> L = Lt[e];
                cpx<T> p1 = tP1[ti], p2 = tP2[ti];
                lds[li] = cmulc(L, p1 - p2) + cmulc(X, p1);
                keep[q] = cmulc(L + X, tE[ti]);
            }
        }
    }
    __syncthreads();
    if constexpr (STAGE == 1 && !LTW)
        lds_fft_held<T, 1>(lds, fc * Ny, Ny, ft, act, ytw);
    else
        lds_fft<T, 1, false>(lds, fc * Ny, Ny, ft, act, twst);
    tile_store<T, NT>(Tt, lds, ne, tid, W, lw, Ny, col0);
    if (STAGE == 2) {
        __syncthreads();
        #pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + q * NT;
            if (e < ne) lds[KZK_LI(e)] = keep[q];
        }
        __syncthreads();
        lds_fft<T, 1, false>(lds, fc * Ny, Ny, ft, act, twst);
        tile_store<T, NT>(Rout + to, lds, ne, tid, W, lw, Ny, col0);
    }
#undef KZK_LI
    if (col0) {
        const T EN = tE[0].x, P1N = tP1[0].x, P2N = tP2[0].x;
        for (int y = tid; y < Ny; y += NT) {
            const long long o = (long long)y * W;
            if (STAGE == 1) {
                const cpx<T> l = It[o];
                Lt[o] = l;
                Tt[o] = cpx<T>{(T)0, P2N * l.y};
            } else {
                const cpx<T> l = Lt[o], m = It[o];
                Tt[o] = cpx<T>{(T)0, (P1N - P2N) * l.y + P1N * m.y};
                Rout[to + o] = cpx<T>{l.x + m.x, EN * (l.y + m.y)};
            }
        }
    }
}

// ------------------------------------------------------------------ multiplier tables (kernel)
template <typename T>
__global__ __launch_bounds__(256) void tables_kernel(const InstDesc* __restrict__ descs, int inst,
                                                     cpx<T>* __restrict__ tabs, int step) {
    // blockIdx.y: column tile m0 = y W; x: position n * W + c within the tile
    const InstDesc& d = descs[inst];
    const int W = d.W, Nh = d.Nh;
    const int rem = blockIdx.x * blockDim.x + threadIdx.x;
    if (rem >= W * Nh) return;
    const int n = rem >> d.log2W, c = rem & (W - 1);
    const int m = (int)blockIdx.y * W + c;
    const long long o = (long long)blockIdx.y * W * Nh + rem;   // storage order
    cpx<T>* tE = tabs + d.off_tab + o;
    cpx<T>* tP1 = tE + d.tab_stride;
    cpx<T>* tP2 = tE + 2 * d.tab_stride;
    if (m == 0) {
        if (n == 0) {   // tau-Nyquist scalars (absorption only), not scaled
            T e, p1, p2;
            nyquist_multipliers<T>(d, e, p1, p2);
            *tE = cpx<T>{e, (T)0};
            *tP1 = cpx<T>{p1, (T)0};
            *tP2 = cpx<T>{p2, (T)0};
        } else {
            *tE = *tP1 = *tP2 = cpx<T>{(T)0, (T)0};
        }
        return;
    }
    mode_multipliers<T>(d, m, n, step, *tE, *tP1, *tP2);
}

// ------------------------------------------------------------------ launchers

template <typename T, int NTT, int MR>
static hipError_t launch_tau_nt(int mode, const InstDesc* d_desc, const TauItem* d_items, int n_items, const T* u_in,
                                T* u_out, const void* Cin, void* Bout, const void* tw, const void* twst, int log2_ntw,
                                int node, int tiled, int prog, unsigned* status, hipStream_t s) {
    dim3 g(n_items), b(NTT);
    const cpx<T>* ci = static_cast<const cpx<T>*>(Cin);
    cpx<T>* bo = static_cast<cpx<T>*>(Bout);
    const cpx<T>* w = static_cast<const cpx<T>*>(tw);
    const cpx<T>* ws = static_cast<const cpx<T>*>(twst);
    switch (mode) {
    case 0: hipLaunchKernelGGL((tau_kernel<T, 0, false, NTT, 0, MR>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, ws, log2_ntw, node, tiled, status); break;
    case 1: hipLaunchKernelGGL((tau_kernel<T, 1, false, NTT, 0, MR>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, ws, log2_ntw, node, tiled, status); break;
    case 2:
        if (prog && tiled)
            hipLaunchKernelGGL((tau_kernel<T, 2, true, NTT, 0, MR>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w,
                               ws, log2_ntw, node, tiled, status);
        else
            hipLaunchKernelGGL((tau_kernel<T, 2, false, NTT, 0, MR>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w,
                               ws, log2_ntw, node, tiled, status);
        break;
    case 3: hipLaunchKernelGGL((tau_kernel<T, 3, false, NTT, 0, MR>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, ws, log2_ntw, node, tiled, status); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int GK>
static hipError_t launch_tau_gen(int mode, const InstDesc* d_desc, const TauItem* d_items, int n_items, const T* u_in,
                                 T* u_out, const void* Cin, void* Bout, const void* tw, int node, int tiled,
                                 unsigned* status, hipStream_t s) {
    dim3 g(n_items), b(TAU_THREADS);
    const cpx<T>* ci = static_cast<const cpx<T>*>(Cin);
    cpx<T>* bo = static_cast<cpx<T>*>(Bout);
    const cpx<T>* w = static_cast<const cpx<T>*>(tw);
    switch (mode) {
    case 0: hipLaunchKernelGGL((tau_kernel<T, 0, false, TAU_THREADS, GK>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, nullptr, 0, node, tiled, status); break;
    case 1: hipLaunchKernelGGL((tau_kernel<T, 1, false, TAU_THREADS, GK>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, nullptr, 0, node, tiled, status); break;
    case 2: hipLaunchKernelGGL((tau_kernel<T, 2, false, TAU_THREADS, GK>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, nullptr, 0, node, tiled, status); break;
    case 3: hipLaunchKernelGGL((tau_kernel<T, 3, false, TAU_THREADS, GK>), g, b, 0, s, d_desc, d_items, u_in, u_out, ci, bo, w, nullptr, 0, node, tiled, status); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool tau_threads_supported(int is_f64, int nt) { return nt == TAU_THREADS || (nt == TAU_THREADS_WIDE && !is_f64); }

template <typename T>
hipError_t launch_tau(int mode, int nt, const InstDesc* d_desc, const TauItem* d_items, int n_items, const T* u_in,
                      T* u_out, const void* Cin, void* Bout, const void* tw, const void* twst, int log2_ntw,
                      int node, int tiled, int prog, int gk, int mr, unsigned* status, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (mr != 3 && mr != 4) return hipErrorInvalidValue;
    if (gk != 0) {
        if (nt != TAU_THREADS) return hipErrorInvalidValue;
        switch (gk) {
        case 4: return launch_tau_gen<T, 4>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw, node, tiled, status, s);
        case 5: return launch_tau_gen<T, 5>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw, node, tiled, status, s);
        case 6: return launch_tau_gen<T, 6>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw, node, tiled, status, s);
        case 7: return launch_tau_gen<T, 7>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw, node, tiled, status, s);
        case 8: return launch_tau_gen<T, 8>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw, node, tiled, status, s);
        case 9: return launch_tau_gen<T, 9>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw, node, tiled, status, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (nt == TAU_THREADS)
        return mr == 4 ? launch_tau_nt<T, TAU_THREADS, 4>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw,
                                                          twst, log2_ntw, node, tiled, prog, status, s)
                       : launch_tau_nt<T, TAU_THREADS, 3>(mode, d_desc, d_items, n_items, u_in, u_out, Cin, Bout, tw,
                                                          twst, log2_ntw, node, tiled, prog, status, s);
    if constexpr (sizeof(T) == 4) {
        if (nt == TAU_THREADS_WIDE)
            return mr == 4 ? launch_tau_nt<T, TAU_THREADS_WIDE, 4>(mode, d_desc, d_items, n_items, u_in, u_out, Cin,
                                                                   Bout, tw, twst, log2_ntw, node, tiled, prog,
                                                                   status, s)
                           : launch_tau_nt<T, TAU_THREADS_WIDE, 3>(mode, d_desc, d_items, n_items, u_in, u_out, Cin,
                                                                   Bout, tw, twst, log2_ntw, node, tiled, prog,
                                                                   status, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int NT, bool FULL, typename S, bool LTW, bool NTL = false>
static hipError_t launch_y_nts(int stage, int ntl, const InstDesc* d_desc, const YItem* d_items, int n_items,
                               int max_blocks, void* C, const void* B, const void* By, void* P, void* U, void* tabs,
                               const void* twst, int step, hipStream_t s) {
    if constexpr (FULL && sizeof(S) == 8 && !NTL) {
        if (ntl)
            return launch_y_nts<T, NT, FULL, S, LTW, true>(stage, ntl, d_desc, d_items, n_items, max_blocks, C, B, By,
                                                           P, U, tabs, twst, step, s);
    }
    dim3 g(max_blocks > 0 && max_blocks < n_items ? max_blocks : n_items), b(NT);
    cpx<T>* c = static_cast<cpx<T>*>(C);
    const cpx<T>* bb = static_cast<const cpx<T>*>(B);
    const cpx<T>* by = static_cast<const cpx<T>*>(By);
    cpx<S>* p = static_cast<cpx<S>*>(P);
    cpx<S>* u = static_cast<cpx<S>*>(U);
    cpx<T>* tb = static_cast<cpx<T>*>(tabs);
    const cpx<T>* ws = static_cast<const cpx<T>*>(twst);
    if (stage == 0)
        hipLaunchKernelGGL((y_kernel<T, NT, 0, FULL, S, LTW, NTL>), g, b, 0, s, d_desc, d_items, n_items, c, bb, by, p, u, tb,
                           ws, step);
    else if (stage == 1)
        hipLaunchKernelGGL((y_kernel<T, NT, 1, FULL, S, LTW, NTL>), g, b, 0, s, d_desc, d_items, n_items, c, bb, by, p, u, tb,
                           ws, step);
    else
        hipLaunchKernelGGL((y_kernel<T, NT, 2, FULL, S, LTW, NTL>), g, b, 0, s, d_desc, d_items, n_items, c, bb, by, p, u, tb,
                           ws, step);
    return hipGetLastError();
}

// s64: FP32 plan with the state in FP64
template <typename T, int NT, bool FULL, bool LTW>
static hipError_t launch_y_nt(int stage, int s64, int ntl, const InstDesc* d_desc, const YItem* d_items, int n_items,
                              int max_blocks, void* C, const void* B, const void* By, void* P, void* U, void* tabs,
                              const void* twst, int step, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (s64)
            return launch_y_nts<T, NT, FULL, double, LTW>(stage, ntl, d_desc, d_items, n_items, max_blocks, C, B, By,
                                                          P, U, tabs, twst, step, s);
    }
    return launch_y_nts<T, NT, FULL, T, LTW>(stage, ntl, d_desc, d_items, n_items, max_blocks, C, B, By, P, U, tabs,
                                             twst, step, s);
}

// full: 0 general tiles, 1 full tiles, 2 full tiles with an 8192-row instance
template <typename T, int NT, typename S>
static int y_resident_nt(int device, int full) {
    int ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu <= 0)
        return 0;
    int lo = 1 << 30;
    // the 8192-row variant exists for blocks of 512 and 1024 threads only;
    // FP32 general tiles load their twiddles per stage
    constexpr bool big = NT >= 512;
    constexpr bool gl = sizeof(T) == 4;
    const void* fns[3][3] = {{(const void*)y_kernel<T, NT, 0, false, S, gl>,
                              (const void*)y_kernel<T, NT, 1, false, S, gl>,
                              (const void*)y_kernel<T, NT, 2, false, S, gl>},
                             {(const void*)y_kernel<T, NT, 0, true, S>, (const void*)y_kernel<T, NT, 1, true, S>,
                              (const void*)y_kernel<T, NT, 2, true, S>},
                             {(const void*)y_kernel<T, NT, 0, true, S, big>,
                              (const void*)y_kernel<T, NT, 1, true, S, big>,
                              (const void*)y_kernel<T, NT, 2, true, S, big>}};
    if (full < 0 || full > 2 || (full == 2 && !big)) return 0;
    for (const void* f : fns[full]) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, NT, 0) != hipSuccess || per <= 0) return 0;
        lo = per < lo ? per : lo;
    }
    return ncu * lo;
}

int y_resident_blocks(int is_f64, int s64, int nt, int full, int device) {
    if (is_f64) {
        switch (nt) {
        case 256: return y_resident_nt<double, 256, double>(device, full);
        case 512: return y_resident_nt<double, 512, double>(device, full);
        default: return 0;
        }
    }
    switch (nt) {
    case 256: return s64 ? y_resident_nt<float, 256, double>(device, full) : y_resident_nt<float, 256, float>(device, full);
    case 512: return s64 ? y_resident_nt<float, 512, double>(device, full) : y_resident_nt<float, 512, float>(device, full);
    case 1024:
        return s64 ? y_resident_nt<float, 1024, double>(device, full) : y_resident_nt<float, 1024, float>(device, full);
    default: return 0;
    }
}

bool y_threads_supported(int is_f64, int nt) {
    if (nt == 256 || nt == 512) return true;
    return nt == 1024 && !is_f64;
}

template <typename T, bool FULL, bool LTW>
static hipError_t launch_y_full(int stage, int s64, int ntl, int nt, const InstDesc* d_desc, const YItem* d_items,
                                int n_items, int max_blocks, void* C, const void* B, const void* By, void* P, void* U,
                                void* tabs, const void* twst, int step, hipStream_t s) {
    switch (nt) {
    case 256:
        if constexpr (!(FULL && LTW))
            return launch_y_nt<T, 256, FULL, LTW>(stage, s64, ntl, d_desc, d_items, n_items, max_blocks, C, B, By, P,
                                                  U, tabs, twst, step, s);
        return hipErrorInvalidValue;
    case 512:
        return launch_y_nt<T, 512, FULL, LTW>(stage, s64, ntl, d_desc, d_items, n_items, max_blocks, C, B, By, P, U,
                                              tabs, twst, step, s);
    case 1024:
        if constexpr (sizeof(T) == 4)
            return launch_y_nt<T, 1024, FULL, LTW>(stage, s64, ntl, d_desc, d_items, n_items, max_blocks, C, B, By, P,
                                                   U, tabs, twst, step, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_y(int stage, int s64, int ntl, int nt, int full, const InstDesc* d_desc, const YItem* d_items,
                    int n_items, int max_blocks, void* C, const void* B, const void* By, void* P, void* U, void* tabs,
                    const void* twst, int step, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (full == 2)
        return launch_y_full<T, true, true>(stage, s64, ntl, nt, d_desc, d_items, n_items, max_blocks, C, B, By, P,
                                            U, tabs, twst, step, s);
    return full ? launch_y_full<T, true, false>(stage, s64, ntl, nt, d_desc, d_items, n_items, max_blocks, C, B, By,
                                                P, U, tabs, twst, step, s)
                : launch_y_full<T, false, sizeof(T) == 4>(stage, s64, ntl, nt, d_desc, d_items, n_items, max_blocks,
                                                          C, B, By, P, U, tabs, twst, step, s);
}

// b^ = sigma F^ in place on one instance's tiled tau-spectrum (element e of
// the instance: tile e / (W n_y), column e mod W, so tau-mode
// m = (e / (W n_y)) W + e mod W; slot m = 0 holds (DC, Nyquist)).
template <typename T>
__global__ __launch_bounds__(256) void flux_diff_kernel(const InstDesc* __restrict__ descs, int inst,
                                                        cpx<T>* __restrict__ X, const cpx<T>* __restrict__ Y) {
    const InstDesc& d = descs[inst];
    const long long n = (long long)d.M * d.n_y, tile = (long long)d.W * d.n_y;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int m = (int)((e / tile) * d.W + (e & (d.W - 1)));
        cpx<T>& x = X[d.off_state + e];
        cpx<T> r = m == 0 ? cpx<T>{(T)0, (T)(-2.0 / d.dtau) * x.y} : cmul(flux_diff_symbol<T>(d, m), x);
        if (Y) r = r + Y[d.off_state + e];
        x = r;
    }
}

template <typename T>
hipError_t launch_flux_diff(const InstDesc* d_desc, int inst, long long n, void* X, const void* Y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 255) / 256;
    dim3 g((unsigned)(blocks < 4096 ? blocks : 4096)), b(256);
    hipLaunchKernelGGL((flux_diff_kernel<T>), g, b, 0, s, d_desc, inst, static_cast<cpx<T>*>(X),
                       static_cast<const cpx<T>*>(Y));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dc(int stage, const InstDesc* d_desc, int n_inst, void* C, void* P, void* U, const void* By,
                     const void* twst, int step, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    cpx<T>* c = static_cast<cpx<T>*>(C);
    cpx<T>* p = static_cast<cpx<T>*>(P);
    cpx<T>* u = static_cast<cpx<T>*>(U);
    const cpx<T>* b = static_cast<const cpx<T>*>(By);
    const cpx<T>* w = static_cast<const cpx<T>*>(twst);
    if (stage == 1)
        hipLaunchKernelGGL((dc_kernel<T, 1>), dim3(n_inst), dim3(512), 0, s, d_desc, c, p, u, b, w, step);
    else
        hipLaunchKernelGGL((dc_kernel<T, 2>), dim3(n_inst), dim3(512), 0, s, d_desc, c, p, u, b, w, step);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_yweno(const InstDesc* d_desc, const YwItem* d_items, int n_items, const T* u, T* by, int node,
                        unsigned* status, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL((yweno_kernel<T>), dim3(n_items), dim3(YW_THREADS), 0, s, d_desc, d_items, u, by, node, status);
    return hipGetLastError();
}

hipError_t launch_velocity(const InstDesc* d_desc, int inst, const double* modes, int n_modes, double x0, double h,
                           int n_nodes, double* tab, double* amax, hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    // the host passes n_y through the descriptor; 8192 rows at most
    hipLaunchKernelGGL(velocity_kernel, dim3(32, n_nodes), dim3(256), 0, s, d_desc, inst, modes, n_modes, x0, h, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(velocity_max_kernel, dim3(n_nodes), dim3(256), 0, s, d_desc, inst, tab, amax);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tables(const InstDesc* d_desc, int inst, int per_tile, int n_tiles, void* tabs, int step,
                         hipStream_t s) {
    if (per_tile <= 0 || n_tiles <= 0) return hipSuccess;
    dim3 g((per_tile + 255) / 256, n_tiles), b(256);
    hipLaunchKernelGGL((tables_kernel<T>), g, b, 0, s, d_desc, inst, static_cast<cpx<T>*>(tabs), step);
    return hipGetLastError();
}

template <typename T, int GK>
static hipError_t launch_tau_adj_gk(int stage, const InstDesc* d_desc, const TauItem* d_items, int n_items,
                                    const void* Tin, const void* Rin, const T* ustore, void* out, const void* tw,
                                    const void* twst, int log2_ntw, int node, unsigned* status, hipStream_t s) {
    dim3 g(n_items), b(TAU_THREADS);
    const cpx<T>* ti = static_cast<const cpx<T>*>(Tin);
    const cpx<T>* ri = static_cast<const cpx<T>*>(Rin);
    cpx<T>* o = static_cast<cpx<T>*>(out);
    const cpx<T>* w = static_cast<const cpx<T>*>(tw);
    const cpx<T>* ws = static_cast<const cpx<T>*>(twst);
    if (stage == 1)
        hipLaunchKernelGGL((tau_adj_kernel<T, 1, GK>), g, b, 0, s, d_desc, d_items, ti, ri, ustore, o, w, ws, log2_ntw, node, status);
    else
        hipLaunchKernelGGL((tau_adj_kernel<T, 2, GK>), g, b, 0, s, d_desc, d_items, ti, ri, ustore, o, w, ws, log2_ntw, node, status);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tau_adj(int stage, const InstDesc* d_desc, const TauItem* d_items, int n_items, const void* Tin,
                          const void* Rin, const T* ustore, void* out, const void* tw, const void* twst,
                          int log2_ntw, int node, int gk, unsigned* status, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (gk) {
    case 0: return launch_tau_adj_gk<T, 0>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    case 4: return launch_tau_adj_gk<T, 4>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    case 5: return launch_tau_adj_gk<T, 5>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    case 6: return launch_tau_adj_gk<T, 6>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    case 7: return launch_tau_adj_gk<T, 7>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    case 8: return launch_tau_adj_gk<T, 8>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    case 9: return launch_tau_adj_gk<T, 9>(stage, d_desc, d_items, n_items, Tin, Rin, ustore, out, tw, twst, log2_ntw, node, status, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int NT, bool LTW>
static hipError_t launch_y_adj_nt(int stage, const InstDesc* d_desc, const YItem* d_items, int n_items, const void* In,
                                  void* Lh, void* Tout, void* Rout, const void* tabs, const void* twst, hipStream_t s) {
    dim3 g(n_items), b(NT);
    const cpx<T>* in = static_cast<const cpx<T>*>(In);
    cpx<T>* lh = static_cast<cpx<T>*>(Lh);
    cpx<T>* to = static_cast<cpx<T>*>(Tout);
    cpx<T>* ro = static_cast<cpx<T>*>(Rout);
    const cpx<T>* tb = static_cast<const cpx<T>*>(tabs);
    const cpx<T>* ws = static_cast<const cpx<T>*>(twst);
    if (stage == 1)
        hipLaunchKernelGGL((y_adj_kernel<T, NT, 1, LTW>), g, b, 0, s, d_desc, d_items, in, lh, to, ro, tb, ws);
    else
        hipLaunchKernelGGL((y_adj_kernel<T, NT, 2, LTW>), g, b, 0, s, d_desc, d_items, in, lh, to, ro, tb, ws);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_y_adj(int stage, int nt, bool big, const InstDesc* d_desc, const YItem* d_items, int n_items,
                        const void* In, void* Lh, void* Tout, void* Rout, const void* tabs, const void* twst,
                        hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (big) {   // n_y = 8192 fills 512 threads per column
        switch (nt) {
        case 512:
            return launch_y_adj_nt<T, 512, true>(stage, d_desc, d_items, n_items, In, Lh, Tout, Rout, tabs, twst, s);
        case 1024:
            if constexpr (sizeof(T) == 4)
                return launch_y_adj_nt<T, 1024, true>(stage, d_desc, d_items, n_items, In, Lh, Tout, Rout, tabs,
                                                      twst, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    }
    switch (nt) {
    case 256: return launch_y_adj_nt<T, 256, false>(stage, d_desc, d_items, n_items, In, Lh, Tout, Rout, tabs, twst, s);
    case 512: return launch_y_adj_nt<T, 512, false>(stage, d_desc, d_items, n_items, In, Lh, Tout, Rout, tabs, twst, s);
    case 1024:
        if constexpr (sizeof(T) == 4)
            return launch_y_adj_nt<T, 1024, false>(stage, d_desc, d_items, n_items, In, Lh, Tout, Rout, tabs, twst,
                                                   s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

int stage_twiddle_entries() { return CT_TABLE_SIZE; }

void stage_twiddles(double* out) {
    for (int MR = 4; MR >= 3; --MR)
        for (int LN = CT_MIN_LN; LN <= CT_MAX_LN; ++LN) {
            int lg = 0;
            while (lg < LN) {
                const int lr = ct_radix(LN, lg, MR);
                if (lg > 0) {
                    const int off = ct_stage_offset(LN, lg, MR), Ns = 1 << lg, R = 1 << lr;
                    for (int kk = 0; kk < Ns; ++kk)
                        for (int s = 0; s < R; ++s) {
                            const double a = -2.0 * KZK_PI * (double)(kk * s) / (double)(Ns * R);
                            out[2 * (off + s * Ns + kk)] = cos(a);
                            out[2 * (off + s * Ns + kk) + 1] = sin(a);
                        }
                }
                lg += lr;
            }
        }
}

#define KZK_INSTANTIATE(T)                                                                                          \
    template hipError_t launch_tau<T>(int, int, const InstDesc*, const TauItem*, int, const T*, T*, const void*,    \
                                      void*, const void*, const void*, int, int, int, int, int, int, unsigned*,     \
                                      hipStream_t);                                                                 \
    template hipError_t launch_y<T>(int, int, int, int, int, const InstDesc*, const YItem*, int, int, void*,        \
                                    const void*, const void*, void*, void*, void*, const void*, int, hipStream_t);   \
    template hipError_t launch_tables<T>(const InstDesc*, int, int, int, void*, int, hipStream_t);                   \
    template hipError_t launch_flux_diff<T>(const InstDesc*, int, long long, void*, const void*, hipStream_t);       \
    template hipError_t launch_dc<T>(int, const InstDesc*, int, void*, void*, void*, const void*, const void*, int,   \
                                     hipStream_t);                                                                   \
    template hipError_t launch_yweno<T>(const InstDesc*, const YwItem*, int, const T*, T*, int, unsigned*,           \
                                        hipStream_t);                                                                \
    template hipError_t launch_tau_adj<T>(int, const InstDesc*, const TauItem*, int, const void*, const void*,      \
                                          const T*, void*, const void*, const void*, int, int, int, unsigned*,       \
                                          hipStream_t);                                                              \
    template hipError_t launch_y_adj<T>(int, int, bool, const InstDesc*, const YItem*, int, const void*, void*,     \
                                        void*, void*, const void*, const void*, hipStream_t);
KZK_INSTANTIATE(float)
KZK_INSTANTIATE(double)
#undef KZK_INSTANTIATE

}  // namespace kzk
