// fft.hpp -- device-side FFT building blocks for gfx950.
//
// Complex arithmetic, radix-2/4/8/16 DFTs held in registers, and Stockham
// autosort stages over data staged in LDS.  Twiddle tables are built in FP64
// on the host and stored in the working precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kzk {

template <typename T> struct alignas(2 * sizeof(T)) cpx { T x, y; };

template <typename T> __device__ __forceinline__ cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T> __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// multiply by S*i (S = +1 or -1)
template <int S, typename T> __device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
    return S > 0 ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------- register DFTs
// X_k = sum_s v_s exp(S 2 pi i s k / R), in place, natural order in and out.

template <typename T, int S> __device__ __forceinline__ void dft2(cpx<T>& a, cpx<T>& b) {
    cpx<T> t = a;
    a = t + b;
    b = t - b;
}

template <typename T, int S> __device__ __forceinline__ void dft4(cpx<T>& v0, cpx<T>& v1, cpx<T>& v2, cpx<T>& v3) {
    cpx<T> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = mul_si<S>(v1 - v3);
    v0 = t0 + t2;
    v2 = t0 - t2;
    v1 = t1 + t3;
    v3 = t1 - t3;
}

template <typename T, int R, int S> struct Dft;

template <typename T, int S> struct Dft<T, 2, S> {
    static __device__ __forceinline__ void run(cpx<T>* v) { dft2<T, S>(v[0], v[1]); }
};
template <typename T, int S> struct Dft<T, 4, S> {
    static __device__ __forceinline__ void run(cpx<T>* v) { dft4<T, S>(v[0], v[1], v[2], v[3]); }
};
template <typename T, int S> struct Dft<T, 8, S> {
    // 8 = 2 x 4: two length-4 DFTs of the even and odd samples, then radix-2.
    static __device__ __forceinline__ void run(cpx<T>* v) {
        const T r = (T)0.70710678118654752440;
        dft4<T, S>(v[0], v[2], v[4], v[6]);
        dft4<T, S>(v[1], v[3], v[5], v[7]);
        // odd part times exp(S 2 pi i k / 8), k = 0..3
        cpx<T> o1 = cmul(v[3], cpx<T>{r, (T)S * r});
        cpx<T> o2 = mul_si<S>(v[5]);
        cpx<T> o3 = cmul(v[7], cpx<T>{-r, (T)S * r});
        cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        v[0] = e0 + v[1]; v[4] = e0 - v[1];
        v[1] = e1 + o1;   v[5] = e1 - o1;
        v[2] = e2 + o2;   v[6] = e2 - o2;
        v[3] = e3 + o3;   v[7] = e3 - o3;
    }
};
template <typename T, int S> struct Dft<T, 16, S> {
    // 16 = 4 x 4: X[k1 + 4 k2] = sum_n2 w16^(n2 k1) [sum_n1 v[4 n1 + n2] w4^(n1 k1)] w4^(n2 k2)
    static __device__ __forceinline__ void run(cpx<T>* v) {
        const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
        const T r = (T)0.70710678118654752440;
        #pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) dft4<T, S>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
        // now v[n2 + 4 k1] = A_{n2}[k1]; twiddle by w16^(n2 k1), w16 = exp(S 2 pi i / 16)
        v[5]  = cmul(v[5],  cpx<T>{c1, (T)S * s1});   // n2=1,k1=1
        v[9]  = cmul(v[9],  cpx<T>{r, (T)S * r});     // n2=1,k1=2
        v[13] = cmul(v[13], cpx<T>{s1, (T)S * c1});   // n2=1,k1=3
        v[6]  = cmul(v[6],  cpx<T>{r, (T)S * r});     // n2=2,k1=1
        v[10] = mul_si<S>(v[10]);                     // n2=2,k1=2
        v[14] = cmul(v[14], cpx<T>{-r, (T)S * r});    // n2=2,k1=3
        v[7]  = cmul(v[7],  cpx<T>{s1, (T)S * c1});   // n2=3,k1=1
        v[11] = cmul(v[11], cpx<T>{-r, (T)S * r});    // n2=3,k1=2
        v[15] = cmul(v[15], cpx<T>{-c1, (T)(-S) * s1}); // n2=3,k1=3: w^9 = -conj-ish
        #pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) dft4<T, S>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        // v[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4x4 index
        cpx<T> t;
        t = v[1]; v[1] = v[4]; v[4] = t;
        t = v[2]; v[2] = v[8]; v[8] = t;
        t = v[3]; v[3] = v[12]; v[12] = t;
        t = v[6]; v[6] = v[9]; v[9] = t;
        t = v[7]; v[7] = v[13]; v[13] = t;
        t = v[11]; v[11] = v[14]; v[14] = t;
    }
};

template <typename T, int S> struct Dft<T, 7, S> {
    // With a_s = v_s + v_{7-s} and b_s = v_s - v_{7-s} (s = 1, 2, 3):
    //   X_k     = v_0 + sum_s cos(2 pi s k / 7) a_s + S i sum_s sin(2 pi s k / 7) b_s,
    //   X_{7-k} = the same with -S,  k = 1, 2, 3;  X_0 = v_0 + a_1 + a_2 + a_3.
    // cos/sin(2 pi m / 7) for m = 1, 2, 3; the products s k reduce mod 7 to
    // these with the signs below (sin(2 pi (7 - m) / 7) = -sin(2 pi m / 7)).
    static __device__ __forceinline__ void run(cpx<T>* v) {
        const T C1 = (T)0.62348980185873353053, C2 = (T)-0.22252093395631440429, C3 = (T)-0.90096886790241912624;
        const T S1 = (T)0.78183148246802980871, S2 = (T)0.97492791218182360702, S3 = (T)0.43388373911755812048;
        const cpx<T> a1 = v[1] + v[6], a2 = v[2] + v[5], a3 = v[3] + v[4];
        const cpx<T> b1 = v[1] - v[6], b2 = v[2] - v[5], b3 = v[3] - v[4];
        const cpx<T> x0 = v[0];
        // k = 1: (C1, C2, C3), (S1, S2, S3); k = 2: (C2, C3, C1), (S2, -S3, -S1); k = 3: (C3, C1, C2), (S3, -S1, S2)
        const cpx<T> c1 = x0 + C1 * a1 + C2 * a2 + C3 * a3, s1 = S1 * b1 + S2 * b2 + S3 * b3;
        const cpx<T> c2 = x0 + C2 * a1 + C3 * a2 + C1 * a3, s2 = S2 * b1 - S3 * b2 - S1 * b3;
        const cpx<T> c3 = x0 + C3 * a1 + C1 * a2 + C2 * a3, s3 = S3 * b1 - S1 * b2 + S2 * b3;
        v[0] = x0 + a1 + a2 + a3;
        const cpx<T> i1 = mul_si<S>(s1), i2 = mul_si<S>(s2), i3 = mul_si<S>(s3);
        v[1] = c1 + i1; v[6] = c1 - i1;
        v[2] = c2 + i2; v[5] = c2 - i2;
        v[3] = c3 + i3; v[4] = c3 - i3;
    }
};

// ---------------------------------------------------------------- twiddles
// w(k) = exp(S 2 pi i k / Ntw) from tw[k] = exp(-2 pi i k / Ntw).
template <int S, typename T> __device__ __forceinline__ cpx<T> twiddle(const cpx<T>* __restrict__ tw, int k) {
    cpx<T> w = tw[k];
    return S > 0 ? cpx<T>{w.x, -w.y} : w;
}

// ---------------------------------------------------------------- LDS layout
// Logical LDS index -> physical slot: one pad slot after every 16 complex
// values, so that accesses at a stride of 16 (the first Stockham stage, and
// the y-pass tiles) spread over all banks instead of hitting one.
__device__ __forceinline__ int padi(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded(int n) { return n + n / 16; }

// ---------------------------------------------------------------- Stockham stages
// A length-n transform (n = 2^LN, 16 <= n <= 8192) at logical LDS positions
// base + idx (base a multiple of 16), done by n/16 threads t, each holding 16
// elements per stage.  Radix schedule MR (log2 of the largest radix): stages
// of radix 2^MR first (MR = 4: radix 16; MR = 3: radix 8, two butterflies per
// thread), then one tail stage of a smaller power of two.  Stage sizes are
// compile-time, so every LDS access of a thread is one padded base address
// plus an immediate offset.  A stage reads the inputs of all its
// butterflies, waits, then writes the outputs (in place).  Twiddles of the
// stage with span Ns*R come from a per-stage table
// twst[off + s*Ns + k] = exp(-2 pi i k s / (Ns R)) (k < Ns, s < R), s-major so
// that the lanes of a wave (consecutive k) read consecutive entries; the
// table holds the stages of every length of the MR = 4 schedule, then those
// of the MR = 3 schedule.

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

constexpr int CT_MIN_LN = 4, CT_MAX_LN = 13;

// radix (log2) of the stage starting at Ns = 2^LG of a length-2^LN transform
__host__ __device__ constexpr int ct_radix(int LN, int LG, int MR = 4) { return (LN - LG) >= MR ? MR : (LN - LG); }

// sum of Ns*R over the stages with Ns > 1 of a length-2^LN transform
__host__ __device__ constexpr int ct_stage_span_sum(int LN, int MR = 4) {
    int tot = 0, lg = 0;
    while (lg < LN) {
        const int lr = ct_radix(LN, lg, MR);
        if (lg > 0) tot += 1 << (lg + lr);
        lg += lr;
    }
    return tot;
}
// entries of the stages of all lengths 2^4 .. 2^13 of one schedule
__host__ __device__ constexpr int ct_schedule_size(int MR) {
    int o = 0;
    for (int l = CT_MIN_LN; l <= CT_MAX_LN; ++l) o += ct_stage_span_sum(l, MR);
    return o;
}
// offset of the stage starting at Ns = 2^LG (schedule MR) in the table
__host__ __device__ constexpr int ct_stage_offset(int LN, int LG, int MR = 4) {
    int o = MR == 4 ? 0 : ct_schedule_size(4);
    for (int l = CT_MIN_LN; l < LN; ++l) o += ct_stage_span_sum(l, MR);
    int lg = 0;
    while (lg < LG) {
        const int lr = ct_radix(LN, lg, MR);
        if (lg > 0) o += 1 << (lg + lr);
        lg += lr;
    }
    return o;
}
constexpr int CT_TABLE_SIZE = ct_schedule_size(4) + ct_schedule_size(3);

// The twiddles a thread needs in the stage starting at Ns = 2^LG: PER blocks
// of R - 1 values (at most 15), w[b * (R - 1) + s - 1] for s = 1 .. R-1.
template <typename T, int S, int LN, int LG, int MR = 4>
__device__ __forceinline__ void ct_fetch(const cpx<T>* __restrict__ twst, int t, bool active, cpx<T> (&w)[15]) {
    if constexpr (LG > 0 && LG < LN) {
        constexpr int LR = ct_radix(LN, LG, MR), R = 1 << LR, PER = 16 / R, tpr = (1 << LN) >> 4, Ns = 1 << LG;
        // every thread loads (the index is in range for any t): a load under a
        // branch would make the compiler wait for it at the branch's join
        (void)active;
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            const cpx<T>* p = twst + ct_stage_offset(LN, LG, MR) + ((t + b * tpr) & (Ns - 1));
            #pragma unroll
            for (int s = 1; s < R; ++s) w[b * (R - 1) + s - 1] = twiddle<S>(p, s * Ns);
        }
    }
}

// Where a stage's twiddles come from.  TW_OWN: the stage requests them
// (into wc) before its LDS reads and barrier.  TW_AHEAD: they are already in
// wc and the stage requests those of the following stage first (into wn), so
// that their latency is covered by this stage's work.  TW_HELD: wc holds the
// forward (S = -1) twiddles for the whole transform, loaded once by the
// caller; an inverse transform multiplies by their conjugates.
enum { TW_OWN = 0, TW_AHEAD = 1, TW_HELD = 2 };

template <typename T, int S, int TW, int LN, int LG, int LR, int MR = 4>
__device__ __forceinline__ void ct_stage(cpx<T>* buf, int base, int t, bool active, const cpx<T>* __restrict__ twst,
                                         cpx<T> (&wc)[15], cpx<T> (&wn)[15]) {
    constexpr int n = 1 << LN, tpr = n >> 4, R = 1 << LR, PER = 16 / R, nR = n / R, Ns = 1 << LG;
    if constexpr (TW == TW_AHEAD)
        ct_fetch<T, S, LN, LG + LR, MR>(twst, t, active, wn);
    else if constexpr (TW == TW_OWN)
        ct_fetch<T, S, LN, LG, MR>(twst, t, active, wc);
    cpx<T> v[PER][R];
    if (active) {
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int j = t + b * tpr;
            if constexpr (nR % 16 == 0) {
                const int p = padi(base + j);
                #pragma unroll
                for (int s = 0; s < R; ++s) v[b][s] = buf[p + 17 * s * (nR / 16)];
            } else {
                #pragma unroll
                for (int s = 0; s < R; ++s) v[b][s] = buf[padi(base + j + s * nR)];
            }
        }
    }
    __syncthreads();
    if (active) {
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int j = t + b * tpr;
            const int k = j & (Ns - 1);
            if constexpr (Ns > 1) {
                #pragma unroll
                for (int s = 1; s < R; ++s)
                    v[b][s] = (TW == TW_HELD && S > 0) ? cmulc(v[b][s], wc[b * (R - 1) + s - 1])
                                                       : cmul(v[b][s], wc[b * (R - 1) + s - 1]);
            }
            Dft<T, R, S>::run(v[b]);
            if constexpr (Ns == 1) {
                // j R .. j R + R - 1 lie in one run of 16 slots (R divides 16)
                static_assert(R >= 8 && R <= 16, "first stage is radix 16 or 8");
                const int p = padi(base + j * R);
                #pragma unroll
                for (int s = 0; s < R; ++s) buf[p + s] = v[b][s];
            } else if constexpr (Ns % 16 == 0) {
                const int p = padi(base + (j - k) * R + k);
                #pragma unroll
                for (int s = 0; s < R; ++s) buf[p + 17 * s * (Ns / 16)] = v[b][s];
            } else {
                #pragma unroll
                for (int s = 0; s < R; ++s) buf[padi(base + (j - k) * R + k + s * Ns)] = v[b][s];
            }
        }
    }
    __syncthreads();
}

template <typename T, int S, int TW, int LN, int LG, int MR>
__device__ __forceinline__ void ct_stages(cpx<T>* buf, int base, int t, bool active, const cpx<T>* __restrict__ twst,
                                          cpx<T> (&wc)[15]) {
    if constexpr (LG < LN) {
        constexpr int LR = ct_radix(LN, LG, MR);
        cpx<T> wn[15];
        ct_stage<T, S, TW, LN, LG, LR, MR>(buf, base, t, active, twst, wc, wn);
        ct_stages<T, S, TW, LN, LG + LR, MR>(buf, base, t, active, twst, wn);
    }
}

template <typename T, int S, int TW, int LN, int MR = 4>
__device__ __forceinline__ void ct_fft(cpx<T>* buf, int base, int t, bool active, const cpx<T>* __restrict__ twst) {
    cpx<T> w0[15];   // the first stage (Ns = 1) has no twiddles
    ct_stages<T, S, TW, LN, 0, MR>(buf, base, t, active, twst, w0);
}

// Held twiddles: the stages with Ns > 1 of a length-2^LN transform
// (LN <= 12: at most two of them, w[0] and w[1]).
template <typename T, int LN, int LG, int I>
__device__ __forceinline__ void ct_fetch_held(const cpx<T>* __restrict__ twst, int t, cpx<T> (&w)[2][15]) {
    if constexpr (LG < LN) {
        constexpr int LR = ct_radix(LN, LG);
        if constexpr (LG > 0) {
            static_assert(I < 2, "at most two stages with twiddles");
            ct_fetch<T, -1, LN, LG>(twst, t, true, w[I]);
            ct_fetch_held<T, LN, LG + LR, I + 1>(twst, t, w);
        } else {
            ct_fetch_held<T, LN, LG + LR, I>(twst, t, w);
        }
    }
}

template <typename T, int S, int LN, int LG, int I>
__device__ __forceinline__ void ct_stages_held(cpx<T>* buf, int base, int t, bool active, cpx<T> (&w)[2][15]) {
    if constexpr (LG < LN) {
        constexpr int LR = ct_radix(LN, LG);
        cpx<T> unused[15];
        if constexpr (LG > 0) {
            ct_stage<T, S, TW_HELD, LN, LG, LR>(buf, base, t, active, nullptr, w[I], unused);
            ct_stages_held<T, S, LN, LG + LR, I + 1>(buf, base, t, active, w);
        } else {
            ct_stage<T, S, TW_HELD, LN, LG, LR>(buf, base, t, active, nullptr, unused, unused);
            ct_stages_held<T, S, LN, LG + LR, I>(buf, base, t, active, w);
        }
    }
}

// Load the held twiddles of thread t for a length-n transform (16 <= n <= 4096).
template <typename T>
__device__ __forceinline__ void lds_fft_twiddles(int n, int t, const cpx<T>* __restrict__ twst, cpx<T> (&w)[2][15]) {
    switch (ilog2(n)) {
    case 4: ct_fetch_held<T, 4, 0, 0>(twst, t, w); break;
    case 5: ct_fetch_held<T, 5, 0, 0>(twst, t, w); break;
    case 6: ct_fetch_held<T, 6, 0, 0>(twst, t, w); break;
    case 7: ct_fetch_held<T, 7, 0, 0>(twst, t, w); break;
    case 8: ct_fetch_held<T, 8, 0, 0>(twst, t, w); break;
    case 9: ct_fetch_held<T, 9, 0, 0>(twst, t, w); break;
    case 10: ct_fetch_held<T, 10, 0, 0>(twst, t, w); break;
    case 11: ct_fetch_held<T, 11, 0, 0>(twst, t, w); break;
    default: ct_fetch_held<T, 12, 0, 0>(twst, t, w); break;
    }
}

// In-place length-n FFT (16 <= n <= 4096) with the thread's twiddles held in
// registers (from lds_fft_twiddles for the same n and t).
template <typename T, int S>
__device__ __forceinline__ void lds_fft_held(cpx<T>* buf, int base, int n, int t, bool active, cpx<T> (&w)[2][15]) {
    switch (ilog2(n)) {
    case 4: ct_stages_held<T, S, 4, 0, 0>(buf, base, t, active, w); break;
    case 5: ct_stages_held<T, S, 5, 0, 0>(buf, base, t, active, w); break;
    case 6: ct_stages_held<T, S, 6, 0, 0>(buf, base, t, active, w); break;
    case 7: ct_stages_held<T, S, 7, 0, 0>(buf, base, t, active, w); break;
    case 8: ct_stages_held<T, S, 8, 0, 0>(buf, base, t, active, w); break;
    case 9: ct_stages_held<T, S, 9, 0, 0>(buf, base, t, active, w); break;
    case 10: ct_stages_held<T, S, 10, 0, 0>(buf, base, t, active, w); break;
    case 11: ct_stages_held<T, S, 11, 0, 0>(buf, base, t, active, w); break;
    default: ct_stages_held<T, S, 12, 0, 0>(buf, base, t, active, w); break;
    }
}

// In-place length-n FFT (16 <= n <= 8192, a power of two) of the sequence at
// logical LDS positions base .. base+n-1 (base a multiple of 16), done by the
// threads t < n/16 where `active`; every thread of the block must call it.
// S = -1: forward, S = +1: inverse (unnormalised).  LA: twiddle look-ahead.
// MR: the radix schedule (4: radix-16 stages, 3: radix-8 stages).
template <typename T, int S, bool LA = true, int MR = 4>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int base, int n, int t, bool active,
                                        const cpx<T>* __restrict__ twst) {
    constexpr int TW = LA ? TW_AHEAD : TW_OWN;
    switch (ilog2(n)) {
    case 4: ct_fft<T, S, TW, 4, MR>(buf, base, t, active, twst); break;
    case 5: ct_fft<T, S, TW, 5, MR>(buf, base, t, active, twst); break;
    case 6: ct_fft<T, S, TW, 6, MR>(buf, base, t, active, twst); break;
    case 7: ct_fft<T, S, TW, 7, MR>(buf, base, t, active, twst); break;
    case 8: ct_fft<T, S, TW, 8, MR>(buf, base, t, active, twst); break;
    case 9: ct_fft<T, S, TW, 9, MR>(buf, base, t, active, twst); break;
    case 10: ct_fft<T, S, TW, 10, MR>(buf, base, t, active, twst); break;
    case 11: ct_fft<T, S, TW, 11, MR>(buf, base, t, active, twst); break;
    case 12: ct_fft<T, S, TW, 12, MR>(buf, base, t, active, twst); break;
    default: ct_fft<T, S, TW, 13, MR>(buf, base, t, active, twst); break;
    }
}

// ---------------------------------------------------------------- lengths 7 * 2^K
// In-place length-M FFT, M = 7 * 2^K (4 <= K <= 9), of the sequence at
// logical LDS positions base .. base+M-1, done by the threads t < M/16
// where `active` (every thread of the block must call it).  Stockham
// stages: radix 7 first (span 7, no twiddles), then radix-16 stages, then
// one tail stage of radix 2, 4 or 8 for the rest of 2^K.  A stage with
// M/R butterflies gives thread t the butterflies t + b M/16, b < ceil(16/R)
// (the radix-7 stage: 16/7 per thread, so its third butterfly exists for
// t < M/56 only).  Twiddles exp(S 2 pi i s k / (Ns R)) come from the table
// tw[i] = exp(-2 pi i i / (2M)) at i = s k (2M / (Ns R)) (s k < Ns R, so
// the index is in range for every thread, active or not).
template <typename T, int S, int M, int NS, int R>
__device__ __forceinline__ void gen_stage(cpx<T>* buf, int base, int t, bool active, const cpx<T>* __restrict__ tw) {
    constexpr int tpr = M / 16, NB = M / R, PER = (NB + tpr - 1) / tpr, TS = 2 * M / (NS * R);
    constexpr bool RAGGED = NB % tpr != 0;
    cpx<T> w[PER][R > 1 ? R - 1 : 1];
    if constexpr (NS > 1) {
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            // the index passes through an empty asm statement, so the loads
            // stay in this stage: with every address known at compile time
            // the compiler would otherwise issue the twiddle loads of all
            // stages at the start of the kernel and hold them in registers
            // through the WENO part (170 instead of 111 VGPRs, half the
            // waves per SIMD)
            int k = (t + b * tpr) % NS;
            asm volatile("" : "+v"(k));
            #pragma unroll
            for (int s = 1; s < R; ++s) w[b][s - 1] = twiddle<S>(tw, s * k * TS);
        }
    }
    cpx<T> v[PER][R];
    if (active) {
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int j = t + b * tpr;
            if (RAGGED && j >= NB) continue;
            #pragma unroll
            for (int s = 0; s < R; ++s) v[b][s] = buf[padi(base + j + s * NB)];
        }
    }
    __syncthreads();
    if (active) {
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            const int j = t + b * tpr;
            if (RAGGED && j >= NB) continue;
            const int k = j % NS;
            if constexpr (NS > 1) {
                #pragma unroll
                for (int s = 1; s < R; ++s) v[b][s] = cmul(v[b][s], w[b][s - 1]);
            }
            Dft<T, R, S>::run(v[b]);
            const int o = base + (j - k) * R + k;
            #pragma unroll
            for (int s = 0; s < R; ++s) buf[padi(o + s * NS)] = v[b][s];
        }
    }
    __syncthreads();
}

// the stages after the first: LR2 = log2 of the power of two still to do
template <typename T, int S, int M, int NS, int LR2>
__device__ __forceinline__ void gen_stages(cpx<T>* buf, int base, int t, bool active, const cpx<T>* __restrict__ tw) {
    if constexpr (LR2 > 0) {
        constexpr int LR = LR2 >= 4 ? 4 : LR2;
        gen_stage<T, S, M, NS, 1 << LR>(buf, base, t, active, tw);
        gen_stages<T, S, M, NS * (1 << LR), LR2 - LR>(buf, base, t, active, tw);
    }
}

template <typename T, int S, int K>
__device__ __forceinline__ void gen_fft(cpx<T>* buf, int base, int t, bool active, const cpx<T>* __restrict__ tw) {
    static_assert(K >= 4 && K <= 9, "lengths 7 * 16 .. 7 * 512");
    constexpr int M = 7 << K;
    gen_stage<T, S, M, 1, 7>(buf, base, t, active, tw);
    gen_stages<T, S, M, 7, K>(buf, base, t, active, tw);
}

}  // namespace kzk
