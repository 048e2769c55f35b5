// fft.hpp -- device-side FFT building blocks for gfx950.
//
// Complex arithmetic, radix-2/4/8/16 DFTs held in registers, and one
// Stockham autosort stage over data staged in LDS.  A length-n transform
// (n a power of two, 16 <= n <= 8192) is done by n/16 threads, each of which
// holds exactly 16 elements per stage: one radix-16 butterfly, or several
// butterflies of the smaller tail radix.  Twiddles come from a table
// tw[k] = exp(-2 pi i k / Ntw) built in FP64 on the host and stored in the
// working precision; a stage of span Ns*R reads it with stride Ntw/(Ns*R).
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

// ---------------------------------------------------------------- one Stockham stage
// Length-n transform stored at buf[base + idx * stride].  Thread t (< n/16)
// takes butterflies j = t + b * n/16... for b < 16/R; the stage reads the
// inputs of all its butterflies, waits, then writes the outputs, so the
// transform runs in place.  Every thread of the block must call it (barriers).
template <typename T, int R, int S>
__device__ __forceinline__ void stockham_stage(cpx<T>* buf, int base, int stride, int n, int Ns, int t,
                                               bool active, const cpx<T>* __restrict__ tw, int log2_tw_span) {
    constexpr int PER = 16 / R;
    const int tpr = n >> 4;
    const int nR = n / R;
    cpx<T> v[PER][R];
    if (active) {
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            int j = t + b * tpr;
            #pragma unroll
            for (int s = 0; s < R; ++s) v[b][s] = buf[padi(base + (j + s * nR) * stride)];
        }
    }
    __syncthreads();
    if (active) {
        // span = Ns * R; twiddle exp(S 2 pi i k s / span) = w(k * s * Ntw / span)
        #pragma unroll
        for (int b = 0; b < PER; ++b) {
            int j = t + b * tpr;
            int k = j & (Ns - 1);
            if (Ns > 1) {
                #pragma unroll
                for (int s = 1; s < R; ++s) v[b][s] = cmul(v[b][s], twiddle<S>(tw, (k * s) << log2_tw_span));
            }
            Dft<T, R, S>::run(v[b]);
            int d = (j - k) * R + k;
            #pragma unroll
            for (int s = 0; s < R; ++s) buf[padi(base + (d + s * Ns) * stride)] = v[b][s];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// Full in-place length-n FFT (16 <= n <= 8192) of the sequence at logical
// LDS positions base + idx * stride, done by threads t < n/16 where `active`.
// log2_ntw = log2 of the twiddle table length (>= log2 n).
template <typename T, int S>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int base, int stride, int n, int t, bool active,
                                        const cpx<T>* __restrict__ tw, int log2_ntw) {
    int Ns = 1;
    int lg = 0;   // log2(Ns)
    const int ln = ilog2(n);
    while (Ns < n) {
        int rem = ln - lg;
        if (rem >= 4) {
            stockham_stage<T, 16, S>(buf, base, stride, n, Ns, t, active, tw, log2_ntw - (lg + 4));
            Ns <<= 4; lg += 4;
        } else if (rem == 3) {
            stockham_stage<T, 8, S>(buf, base, stride, n, Ns, t, active, tw, log2_ntw - (lg + 3));
            Ns <<= 3; lg += 3;
        } else if (rem == 2) {
            stockham_stage<T, 4, S>(buf, base, stride, n, Ns, t, active, tw, log2_ntw - (lg + 2));
            Ns <<= 2; lg += 2;
        } else {
            stockham_stage<T, 2, S>(buf, base, stride, n, Ns, t, active, tw, log2_ntw - (lg + 1));
            Ns <<= 1; lg += 1;
        }
    }
}

}  // namespace kzk
