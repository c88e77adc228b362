// Device helpers shared by the polyrecon kernels: complex arithmetic, phasors
// with float64 range reduction, and a mixed-radix Stockham FFT in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace pl {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by +i (sgn = +1) or -i (sgn = -1)
__device__ __forceinline__ float2 cmul_i(float2 a, int sgn) {
    return sgn > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// v broadcast from lane `lane` of the wavefront (wavefront-uniform result).
__device__ __forceinline__ float rdl(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// exp(j 2 pi x) for |x| <= 256 revolutions by the hardware sine and cosine
// (v_sin_f32 / v_cos_f32 take revolutions; measured on gfx950: absolute error
// at most 1.3e-7 over [-8, 8]).
__device__ __forceinline__ float2 cis_rev_f(float x) {
    return make_float2(__builtin_amdgcn_cosf(x), __builtin_amdgcn_sinf(x));
}

// exp(j 2 pi rev): the revolution count is reduced to [-1/2, 1/2] in float64
// before the float32 evaluation, so phases of thousands of radians keep full
// float32 accuracy.
__device__ __forceinline__ float2 cis_rev(double rev) {
    return cis_rev_f(static_cast<float>(rev - rint(rev)));
}

// exp(j phase) for a float64 phase in radians.
__device__ __forceinline__ float2 cis(double phase) { return cis_rev(phase * (0.5 / kPi)); }

// ------------------------------------------------------------ Stockham FFT
// One radix-R butterfly on registers: X_r = sum_q a_q exp(sgn 2 pi i q r / R).
template <int R>
__device__ __forceinline__ void dft_small(float2* a, int sgn);

template <>
__device__ __forceinline__ void dft_small<2>(float2* a, int) {
    const float2 t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
}

template <>
__device__ __forceinline__ void dft_small<4>(float2* a, int sgn) {
    const float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const float2 t2 = cadd(a[1], a[3]), t3 = cmul_i(csub(a[1], a[3]), sgn);
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
}

template <>
__device__ __forceinline__ void dft_small<8>(float2* a, int sgn) {
    // split into even and odd halves, two radix-4 transforms, then combine
    float2 e[4] = {a[0], a[2], a[4], a[6]};
    float2 o[4] = {a[1], a[3], a[5], a[7]};
    dft_small<4>(e, sgn);
    dft_small<4>(o, sgn);
    const float h = 0.70710678118654752f;
    // twiddles exp(sgn 2 pi i q / 8), q = 0..3
    const float2 w1 = make_float2(h, sgn * h);
    o[1] = cmul(o[1], w1);
    o[2] = cmul_i(o[2], sgn);
    o[3] = cmul(o[3], make_float2(-h, sgn * h));
    for (int q = 0; q < 4; ++q) {
        a[q] = cadd(e[q], o[q]);
        a[q + 4] = csub(e[q], o[q]);
    }
}

template <>
__device__ __forceinline__ void dft_small<3>(float2* a, int sgn) {
    const float c = -0.5f, s = 0.86602540378443865f * sgn;
    const float2 t = cadd(a[1], a[2]);
    const float2 u = csub(a[1], a[2]);
    const float2 m = make_float2(a[0].x + c * t.x, a[0].y + c * t.y);
    const float2 v = make_float2(-s * u.y, s * u.x);  // i s u
    a[0] = cadd(a[0], t);
    a[1] = cadd(m, v);
    a[2] = csub(m, v);
}

template <>
__device__ __forceinline__ void dft_small<5>(float2* a, int sgn) {
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float s1 = 0.95105651629515357f * sgn, s2 = 0.58778525229247313f * sgn;
    const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
    const float2 u1 = csub(a[1], a[4]), u2 = csub(a[2], a[3]);
    const float2 m1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
    const float2 m2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
    // i (s1 u1 + s2 u2) and i (s2 u1 - s1 u2)
    const float2 v1 = make_float2(-(s1 * u1.y + s2 * u2.y), s1 * u1.x + s2 * u2.x);
    const float2 v2 = make_float2(-(s2 * u1.y - s1 * u2.y), s2 * u1.x - s1 * u2.x);
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(m1, v1);
    a[4] = csub(m1, v1);
    a[2] = cadd(m2, v2);
    a[3] = csub(m2, v2);
}

// One Stockham stage of radix R over `ntr` transforms of length n stored at
// src[t * ld + i]; writes dst.  tw[j] = exp(-2 pi i j / n).  Ns is the product
// of the radices of the previous stages.
// floor(x / d) for 0 <= x, 1 <= d and x + d < 2^22, from inv_d = 1.0f / d
// (correctly rounded): (x + 1/2) / d = floor(x / d) + f with f in
// [1/(2d), 1 - 1/(2d)], and the float product is within (x + d) 2^-23 / d of
// it, less than 1/(2d).  A few instructions instead of an integer division.
__device__ __forceinline__ int div_small(int x, float inv_d) {
    return static_cast<int>((static_cast<float>(x) + 0.5f) * inv_d);
}

template <int R>
__device__ __forceinline__ void stockham_stage(const float2* __restrict__ src, float2* __restrict__ dst,
                                               int n, int ld, int ntr, int Ns,
                                               const float2* __restrict__ tw, int sgn, int tid,
                                               int nthreads) {
    const int nb = n / R;
    const int tstep = n / (Ns * R);
    const int total = nb * ntr;
    const float inv_nb = 1.0f / nb, inv_ns = 1.0f / Ns;
    for (int b = tid; b < total; b += nthreads) {
        const int t = ntr == 1 ? 0 : div_small(b, inv_nb);
        const int j = b - t * nb;
        const int jq = div_small(j, inv_ns);
        const int k = j - jq * Ns;
        const float2* s = src + t * ld;
        float2 a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = s[j + r * nb];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            float2 w = tw[r * k * tstep];
            if (sgn > 0) w.y = -w.y;
            a[r] = cmul(a[r], w);
        }
        dft_small<R>(a, sgn);
        float2* d = dst + t * ld + jq * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) d[r * Ns] = a[r];
    }
}

// Full transform in LDS; returns the buffer holding the result (a or b).
// Barriers are issued by every thread of the block.
__device__ inline float2* lds_fft(float2* a, float2* b, int n, int ld, int ntr, const Radices& rad,
                                  const float2* __restrict__ tw, int sgn, int tid, int nthreads) {
    int Ns = 1;
    for (int st = 0; st < rad.count; ++st) {
        const int R = rad.r[st];
        switch (R) {
            case 8: stockham_stage<8>(a, b, n, ld, ntr, Ns, tw, sgn, tid, nthreads); break;
            case 4: stockham_stage<4>(a, b, n, ld, ntr, Ns, tw, sgn, tid, nthreads); break;
            case 2: stockham_stage<2>(a, b, n, ld, ntr, Ns, tw, sgn, tid, nthreads); break;
            case 3: stockham_stage<3>(a, b, n, ld, ntr, Ns, tw, sgn, tid, nthreads); break;
            default: stockham_stage<5>(a, b, n, ld, ntr, Ns, tw, sgn, tid, nthreads); break;
        }
        __syncthreads();
        float2* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// ------------------------------------------------ wavefront FFT of 64 R points
// One wavefront transforms N = 64 R values (R 2,3,5-smooth, at most 32)
// held in LDS, with no workgroup barrier: with n = 64 a + l and
// k = k1 + R k2,
//   X[k1 + R k2] = sum_l w64^(l k2) [wN^(l k1) sum_a x[64 a + l] wR^(a k1)]
// (w_M = exp(+2 pi i / M)): lane l takes the R-point DFT over a in
// registers and its twiddles, then the R transforms of 64 points over l
// run as two radix-8 passes through LDS (l = l1 + 8 l2, k2 = m1 + 8 m2).
// Rows of the transposed stages are kWaveRow = 72 complex values apart and
// the middle pass writes its outputs at 9 m1 + l1 in the row, which keeps
// the 8-byte LDS accesses of 32 lanes on distinct banks in every pass.

// exp(+2 pi i j / R) at compile time (angle reduced to [-pi, pi], Taylor
// series in double).
constexpr double ct_angle(int j, int r) {
    int m = j % r;
    if (m < 0) m += r;
    if (2 * m > r) m -= r;
    return 2.0 * kPi * m / r;
}
constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 16; ++n) {
        term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}
constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 16; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
template <int R>
struct RootsOfUnity {
    float re[R], im[R];
    constexpr RootsOfUnity() : re(), im() {
        for (int j = 0; j < R; ++j) {
            re[j] = static_cast<float>(ct_cos(ct_angle(j, R)));
            im[j] = static_cast<float>(ct_sin(ct_angle(j, R)));
        }
    }
};

// the factor a composite R is split by (the first of 8, 4, 2, 3, 5 below R)
constexpr int split_factor(int r) {
    return (r % 8 == 0 && r > 8) ? 8 : (r % 4 == 0 && r > 4) ? 4 : (r % 2 == 0 && r > 2) ? 2 : (r % 3 == 0 && r > 3) ? 3 : 5;
}
constexpr bool is_codelet(int r) { return r == 2 || r == 3 || r == 4 || r == 5 || r == 8; }

// Inverse DFT of R values in registers, natural order in and out.
template <int R>
__device__ __forceinline__ void idft_reg(float2* x) {
    if constexpr (is_codelet(R)) {
        dft_small<R>(x, +1);
    } else {
        constexpr int A = split_factor(R), B = R / A;
        constexpr RootsOfUnity<R> w{};
        float2 t[R];
        // n = n1 + A n2, k = B k1 + k2: B-point DFTs over n2, twiddles
        // wR^(n1 k2), A-point DFTs over n1
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) {
            float2 u[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) u[n2] = x[n1 + A * n2];
            idft_reg<B>(u);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2)
                t[n1 * B + k2] = (n1 * k2) % R == 0
                                     ? u[k2]
                                     : cmul(u[k2], make_float2(w.re[(n1 * k2) % R], w.im[(n1 * k2) % R]));
        }
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            float2 v[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) v[n1] = t[n1 * B + k2];
            idft_reg<A>(v);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) x[B * k1 + k2] = v[k1];
        }
    }
}

// Orders this wavefront's LDS accesses: DS instructions of a wavefront
// complete in issue order, so a compiler barrier suffices.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWaveRow = 72;   // complex values per row of the transposed stages

// Inverse FFT of the N = 64 R values A[0, N) of one wavefront (see above);
// out(k, X[k]) receives every output once.  A is R rows of kWaveRow.
template <int R, typename Out>
__device__ __forceinline__ void wave_ifft(float2* A, const float2* __restrict__ tw, int lane, Out out) {
    // R-point transforms over a, twiddles wN^(l k1), rows k1
    {
        float2 x[R];
#pragma unroll
        for (int j = 0; j < R; ++j) x[j] = A[64 * j + lane];
        idft_reg<R>(x);
#pragma unroll
        for (int k1 = 1; k1 < R; ++k1) {
            const float2 w = tw[lane * k1];   // exp(-2 pi i lane k1 / N), lane k1 < N
            x[k1] = cmul(x[k1], make_float2(w.x, -w.y));
        }
        wave_lds_sync();
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) A[k1 * kWaveRow + lane] = x[k1];
    }
    wave_lds_sync();

    // first radix-8 pass over l2 (butterfly (k1, l1)), twiddles w64^(l1 m1)
    for (int b = lane; b < 8 * R; b += 64) {
        const int k1 = b >> 3, l1 = b & 7;
        float2* row = A + k1 * kWaveRow;
        float2 u[8];
#pragma unroll
        for (int l2 = 0; l2 < 8; ++l2) u[l2] = row[l1 + 8 * l2];
        dft_small<8>(u, +1);
#pragma unroll
        for (int m1 = 1; m1 < 8; ++m1) {
            const float2 w = tw[R * l1 * m1];
            u[m1] = cmul(u[m1], make_float2(w.x, -w.y));
        }
#pragma unroll
        for (int m1 = 0; m1 < 8; ++m1) row[9 * m1 + l1] = u[m1];
    }
    wave_lds_sync();

    // second radix-8 pass over l1 (butterfly (k1, m1)): X[k1 + R (m1 + 8 m2)]
    for (int b = lane; b < 8 * R; b += 64) {
        const int k1 = b >> 3, m1 = b & 7;
        const float2* row = A + k1 * kWaveRow + 9 * m1;
        float2 v[8];
#pragma unroll
        for (int l1 = 0; l1 < 8; ++l1) v[l1] = row[l1];
        dft_small<8>(v, +1);
#pragma unroll
        for (int m2 = 0; m2 < 8; ++m2) out(k1 + R * (m1 + 8 * m2), v[m2]);
    }
}

}  // namespace pl
