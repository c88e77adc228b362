// Plan tables, the batched FFTs over the scan axis (eq. 2/12) and over k_z
// (eq. 9), and twiddle tables.
#include "device.hpp"

namespace pl {
namespace {

struct PlanTablesArgs {
    int n_ch, n_z, n_f, n_l, n_fine, interp, n_gl, block, ref_mode;
    double du, h, beta, scan_step;
    double gx0, gx1, gy0, gy1;
    double kref[kMaxBlocks];
    double glx[kMaxGL];
    double glw[kMaxGL];
};

__device__ double kz_of(int kap, int n_z, double step) {
    const int sk = kap < (n_z + 1) / 2 ? kap : kap - n_z;
    return 2.0 * kPi * sk / (n_z * step);
}

// Reference wavenumber of k_z bin kap (see plan_tables_kernel).
__device__ double kref_of(const PlanTablesArgs& a, const double* __restrict__ k, int kap) {
    if (a.ref_mode != PL_REF_MIN_K) return a.kref[kap / a.block];
    const double q = 0.25 * kz_of(kap, a.n_z, a.scan_step) * kz_of(kap, a.n_z, a.scan_step);
    for (int f = 0; f < a.n_f; ++f) {   // k rises with f: the first real k_rho is the smallest
        const double arg = k[f] * k[f] - q;
        if (arg > 0.0) return sqrt(arg);
    }
    return 0.0;
}

__device__ double dist_to_rect(double px, double py, double x0, double x1, double y0, double y1) {
    const double cx = fmin(fmax(px, x0), x1), cy = fmin(fmax(py, y0), y1);
    return hypot(px - cx, py - cy);
}

// Fills the per-call tables of the hybrid plan:
//   llo[c]       start of channel c's range grid (lowest range over the pixel
//                rectangle minus two steps)
//   lref[c]      range rho_T + rho_R from channel c to the centre of the pixel
//                rectangle (demodulation reference of the resampling method)
//   tw_fine[t]   exp(-2 pi i t / n_fine)
//   deap[i]      1 / (h * FT of the spreading kernel) at output mode i - n_l/2
//   kp[kz][f]    k' = k_rho - k_ref(kz), k_rho = sqrt(k^2 - k_z^2/4) (0 if evanescent)
//   wk[kz][f]    k_f (weight of "k dk") times the B-spline prefilter, 0 if evanescent
//   krz[kz]      the reference k_ref(kz): the block's band centre, or with
//                PL_REF_MIN_K the paper's k_rho0 = k_rho at the lowest
//                wavenumber k[0] (the smallest real k_rho of the bin when
//                k[0] is evanescent there, 0 when nothing propagates)
__global__ void plan_tables_kernel(PlanTablesArgs a, const double* __restrict__ chan,
                                   const double* __restrict__ k, double* __restrict__ llo,
                                   double* __restrict__ lref, float2* __restrict__ tw_fine,
                                   float* __restrict__ deap, double* __restrict__ kp,
                                   float* __restrict__ wk, double* __restrict__ krz) {
    const long long n0 = a.n_ch, n1 = n0 + a.n_z, n2 = n1 + a.n_fine, n3 = n2 + a.n_l;
    const long long total = n3 + static_cast<long long>(a.n_z) * a.n_f;
    for (long long idx = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; idx < total;
         idx += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (idx < n0) {
            const int c = static_cast<int>(idx);
            const double lmin = dist_to_rect(chan[4 * c], chan[4 * c + 1], a.gx0, a.gx1, a.gy0, a.gy1) +
                                dist_to_rect(chan[4 * c + 2], chan[4 * c + 3], a.gx0, a.gx1, a.gy0, a.gy1);
            llo[c] = lmin - 2.0 * a.du;
            const double cx = 0.5 * (a.gx0 + a.gx1), cy = 0.5 * (a.gy0 + a.gy1);
            lref[c] = hypot(cx - chan[4 * c], cy - chan[4 * c + 1]) + hypot(cx - chan[4 * c + 2], cy - chan[4 * c + 3]);
        } else if (idx < n1) {
            const int kap = static_cast<int>(idx - n0);
            krz[kap] = kref_of(a, k, kap);
        } else if (idx < n2) {
            const int t = static_cast<int>(idx - n1);
            double s, c;
            sincospi(-2.0 * t / a.n_fine, &s, &c);
            tw_fine[t] = make_float2(static_cast<float>(c), static_cast<float>(s));
        } else if (idx < n3) {
            const int i = static_cast<int>(idx - n2);
            const double xi = 2.0 * kPi * a.h * (i - a.n_l / 2) / a.n_fine;
            double ft = 0.0;
            for (int q = 0; q < a.n_gl; ++q) {
                const double z = a.glx[q];
                ft += a.glw[q] * exp(a.beta * (sqrt(1.0 - z * z) - 1.0)) * cos(xi * z);
            }
            deap[i] = static_cast<float>(1.0 / (a.h * ft));
        } else {
            const long long e = idx - n3;
            const int kap = static_cast<int>(e / a.n_f), f = static_cast<int>(e % a.n_f);
            const double kz = kz_of(kap, a.n_z, a.scan_step);
            const double arg = k[f] * k[f] - 0.25 * kz * kz;
            const bool valid = arg > 0.0;
            const double kr = valid ? sqrt(arg) : 0.0;
            const double kpr = kr - kref_of(a, k, kap);
            kp[e] = kpr;
            double w = valid ? k[f] : 0.0;
            if (valid && a.interp == PL_INTERP_BSPLINE4) {
                const double x = 0.5 * kpr * a.du;
                const double sinc = fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x;
                w /= (sinc * sinc) * (sinc * sinc);
            }
            wk[e] = static_cast<float>(w);
        }
    }
}

// Tables of an AxisFft (see internal.hpp): tw[t] = exp(-2 pi i t / m); for
// the chirp-z form w[t] = exp(-i pi t^2 / n), t < n, with t^2 reduced mod 2n
// in integers so that the float64 sine and cosine see an argument below 2;
// pad[j] = conj(w[t]) for j = t < n and j = m - t (0 < t < n), else 0 (the
// filter of the cyclic convolution; its transform is taken next).
__global__ void axis_fft_tables_kernel(int n, int m, int chirp, float2* __restrict__ tw, float2* __restrict__ w,
                                       float2* __restrict__ pad) {
    const int total = m + (chirp ? n + m : 0);
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        double s, c;
        if (idx < m) {
            sincospi(-2.0 * idx / m, &s, &c);
            tw[idx] = make_float2(static_cast<float>(c), static_cast<float>(s));
        } else if (idx < m + n) {
            const long long t = idx - m;
            const long long r = (t * t) % (2LL * n);
            sincospi(-static_cast<double>(r) / n, &s, &c);
            w[t] = make_float2(static_cast<float>(c), static_cast<float>(s));
        } else {
            const int j = idx - m - n;
            const long long t = j < n ? j : (j > m - n ? m - j : -1);
            float2 v = make_float2(0.f, 0.f);
            if (t >= 0) {
                const long long r = (t * t) % (2LL * n);
                sincospi(static_cast<double>(r) / n, &s, &c);
                v = make_float2(static_cast<float>(c), static_cast<float>(s));
            }
            pad[j] = v;
        }
    }
}

struct FftArgs {
    int n, m, nbatch, inner, per_wg, ld, sign, n_fast_in, n_fast_out;
    long long in_so, in_si, in_sn, out_so, out_si, out_sn;
    float scale, inv_inner, inv_n, inv_m, inv_pad;   // reciprocals for div_small: 1/inner, 1/n, 1/m, 1/(m - n)
    Radices rad;
};

// Batched FFT of length n along a strided axis.  Batch index b splits into
// (outer o = b / inner, inner s = b % inner); element i of transform b is at
// in[o*in_so + s*in_si + i*in_sn].  Each block transforms per_wg batches in
// LDS (two buffers of per_wg * ld complex values).
__global__ __launch_bounds__(256) void fft_strided_kernel(const float2* __restrict__ in,
                                                          float2* __restrict__ out,
                                                          const float2* __restrict__ tw, FftArgs a) {
    extern __shared__ float2 smem[];
    float2* A = smem;
    float2* B = smem + a.per_wg * a.ld;
    const int b0 = blockIdx.x * a.per_wg;
    const int nb = min(a.per_wg, a.nbatch - b0);
    const int total = nb * a.n;
    const int tid = threadIdx.x;
    for (int e = tid; e < total; e += blockDim.x) {
        int t, i;
        if (a.n_fast_in) {
            t = e / a.n;
            i = e - t * a.n;
        } else {
            i = e / nb;
            t = e - i * nb;
        }
        const int b = b0 + t;
        const int o = b / a.inner, s = b - o * a.inner;
        A[t * a.ld + i] = in[o * a.in_so + s * a.in_si + i * a.in_sn];
    }
    __syncthreads();
    const float2* res = lds_fft(A, B, a.n, a.ld, nb, a.rad, tw, a.sign, tid, blockDim.x);
    for (int e = tid; e < total; e += blockDim.x) {
        int t, i;
        if (a.n_fast_out) {
            t = e / a.n;
            i = e - t * a.n;
        } else {
            i = e / nb;
            t = e - i * nb;
        }
        const int b = b0 + t;
        const int o = b / a.inner, s = b - o * a.inner;
        out[o * a.out_so + s * a.out_si + i * a.out_sn] = cscale(res[t * a.ld + i], a.scale);
    }
}

// Bluestein's chirp-z transform (1970) for lengths that are not 2,3,5-smooth.
// With t k = (t^2 + k^2 - (k - t)^2) / 2 and w[t] = exp(-i pi t^2 / n),
//   X[k] = sum_t x[t] exp(-2 pi i t k / n) = w[k] sum_t (x[t] w[t]) conj(w[k - t]),
// a linear convolution of length 2n - 1, evaluated as a cyclic one of the
// smooth length m >= 2n - 1: forward transform of x w zero-padded to m,
// product with hat = FFT_m(pad) / m, inverse transform, times w[k] for k < n.
// The inverse transform (sign +1) conjugates its input and output.  Each
// block transforms per_wg batches in LDS (two buffers of per_wg * ld values,
// ld = m + 1); batch and element indexing as in fft_strided_kernel.
__global__ __launch_bounds__(256) void fft_chirp_strided_kernel(const float2* __restrict__ in,
                                                                float2* __restrict__ out,
                                                                const float2* __restrict__ tw,
                                                                const float2* __restrict__ w,
                                                                const float2* __restrict__ hat, FftArgs a) {
    extern __shared__ float2 smem[];
    float2* A = smem;
    float2* B = smem + a.per_wg * a.ld;
    const int b0 = blockIdx.x * a.per_wg;
    const int nb = min(a.per_wg, a.nbatch - b0);
    const int tid = threadIdx.x;
    const bool inv = a.sign > 0;
    const float inv_nb = 1.0f / nb;
    const int pad = a.m - a.n;
    for (int e = tid; e < nb * pad; e += blockDim.x) {
        const int t = div_small(e, a.inv_pad);
        A[t * a.ld + a.n + (e - t * pad)] = make_float2(0.f, 0.f);
    }
    const int total = nb * a.n;
    for (int e = tid; e < total; e += blockDim.x) {
        int t, i;
        if (a.n_fast_in) {
            t = div_small(e, a.inv_n);
            i = e - t * a.n;
        } else {
            i = div_small(e, inv_nb);
            t = e - i * nb;
        }
        const int b = b0 + t;
        const int o = div_small(b, a.inv_inner), s = b - o * a.inner;
        float2 v = in[o * a.in_so + s * a.in_si + i * a.in_sn];
        if (inv) v.y = -v.y;
        A[t * a.ld + i] = cmul(v, w[i]);
    }
    __syncthreads();
    float2* r = lds_fft(A, B, a.m, a.ld, nb, a.rad, tw, -1, tid, blockDim.x);
    for (int e = tid; e < nb * a.m; e += blockDim.x) {
        const int t = div_small(e, a.inv_m), i = e - t * a.m;
        r[t * a.ld + i] = cmul(r[t * a.ld + i], hat[i]);
    }
    __syncthreads();
    r = lds_fft(r, r == A ? B : A, a.m, a.ld, nb, a.rad, tw, +1, tid, blockDim.x);
    for (int e = tid; e < total; e += blockDim.x) {
        int t, i;
        if (a.n_fast_out) {
            t = div_small(e, a.inv_n);
            i = e - t * a.n;
        } else {
            i = div_small(e, inv_nb);
            t = e - i * nb;
        }
        const int b = b0 + t;
        const int o = div_small(b, a.inv_inner), s = b - o * a.inner;
        float2 v = cmul(r[t * a.ld + i], w[i]);
        if (inv) v.y = -v.y;
        out[o * a.out_so + s * a.out_si + i * a.out_sn] = cscale(v, a.scale);
    }
}

// Workgroups of 256 threads of `fn` with `smem` bytes of LDS that are
// resident at once on the device, at most `groups`: the grid of a launch
// whose workgroups loop over groups of work.  Returns the count, or minus an
// error code.
int resident_grid(const void* fn, size_t smem, const char* what, long long groups) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1 ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, smem) != hipSuccess)
        return -fail(PL_EDEVICE, "%s: occupancy query failed", what);
    return static_cast<int>(std::max<long long>(1, std::min<long long>(groups, static_cast<long long>(std::max(1, per_cu)) * cus)));
}

// The same batched strided FFT for N = 64 R (R at most 8) on the wavefront
// FFT (wave_ifft): a workgroup stages TB transforms in LDS with loads and
// stores that run along whichever of (transform, element) is contiguous in
// memory (TB = 16: 128-byte runs across transforms), its NW wavefronts
// transform them in place (wave_ifft's last radix-8 pass is a single pass
// for R <= 8, so every lane has read its inputs before any output lands),
// and the forward direction conjugates on the way in and out.  Transforms
// are kWaveRow R + 2 values apart in LDS: 4 dwords of bank offset apiece.
template <int R, int TB, int NW>
__global__ __launch_bounds__(64 * NW) void fft_wave_strided_kernel(const float2* __restrict__ in,
                                                               float2* __restrict__ out,
                                                               const float2* __restrict__ tw, FftArgs a) {
    constexpr int N = 64 * R;
    constexpr int PS = kWaveRow * R + 2;
    extern __shared__ float2 smem[];
    const int b0 = blockIdx.x * TB;
    const int nb = min(TB, a.nbatch - b0);
    const int tid = threadIdx.x;
    const bool fwd = a.sign < 0;
    for (int e = tid; e < TB * N; e += 64 * NW) {
        int t, i;
        if (a.n_fast_in) {
            t = e / N;
            i = e - t * N;
        } else {
            i = e / TB;
            t = e - i * TB;
        }
        if (t < nb) {
            const int b = b0 + t;
            const int o = div_small(b, a.inv_inner), s = b - o * a.inner;
            float2 v = in[o * a.in_so + s * a.in_si + i * a.in_sn];
            if (fwd) v.y = -v.y;
            smem[t * PS + i] = v;
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    for (int t = wave; t < nb; t += NW) {
        float2* A = smem + t * PS;
        wave_ifft<R>(A, tw, lane, [&](int k, float2 v) { A[k] = v; });
    }
    __syncthreads();
    for (int e = tid; e < TB * N; e += 64 * NW) {
        int t, i;
        if (a.n_fast_out) {
            t = e / N;
            i = e - t * N;
        } else {
            i = e / TB;
            t = e - i * TB;
        }
        if (t < nb) {
            const int b = b0 + t;
            const int o = div_small(b, a.inv_inner), s = b - o * a.inner;
            float2 v = smem[t * PS + i];
            if (fwd) v.y = -v.y;
            out[o * a.out_so + s * a.out_si + i * a.out_sn] = cscale(v, a.scale);
        }
    }
}

// Bluestein's chirp-z transform (as fft_chirp_strided_kernel) for a cyclic
// length m = 64 R, one wavefront per transform and no workgroup barrier
// inside a transform.  The forward product is formed through the inverse
// wavefront FFT I (exponent +): DFT(a) = conj(I(conj a)).  I runs as in
// wave_ifft up to its last radix-8 pass, which leaves butterfly (k1, m1) of
// a lane holding Y[k1 + R (m1 + 8 m2)], m2 = 0..7, in registers; the product
// Z = conj(Y) hat is taken there, and the convolution c = I(Z) comes from the
// transpose of the same factorisation (the DFT matrix is symmetric): its
// passes in reverse order take the scrambled index order in and give natural
// order out, lane l holding c[64 a + l].  Transposed passes, with
// n = 64 a + l, l = l1 + 8 l2, k = k1 + R (m1 + 8 m2):
//   over m2 (in registers): sum Z w8^(l1 m2), stored at 9 m1 + l1 of row k1;
//   over m1: twiddle w64^(l1 m1), sum w8^(l2 m1), stored at l of row k1;
//   over k1 (lane l): twiddle wN^(l k1), R-point sum wR^(a k1).
// A workgroup stages TB transforms of n points in LDS (loads and stores as
// in fft_wave_strided_kernel) beside the twiddles, the chirp and the filter
// (read once per workgroup); each wavefront has R rows of kWaveRow values of
// its own for the passes.
int set_lds_limit(const void* fn, size_t smem, const char* what);

template <int R, int TB>
__global__ __launch_bounds__(256) void fft_chirp_wave_kernel(const float2* __restrict__ in, float2* __restrict__ out,
                                                             const float2* __restrict__ tw,
                                                             const float2* __restrict__ w,
                                                             const float2* __restrict__ hat, FftArgs a) {
    static_assert(R >= 2 && R <= 32, "cyclic lengths of 128 to 2048 points");
    constexpr int N = 64 * R;
    extern __shared__ float2 smem[];
    const int PS = a.n | 1;                         // staged transform stride (odd)
    float2* const stage = smem;                     // [TB][PS]
    float2* const ltw = smem + ((TB * PS + 1) & ~1);   // twiddles [N], filter [N], chirp [n]
    float2* const lhat = ltw + N;
    float2* const lw = lhat + N;
    const int tid = threadIdx.x;
    const bool inv = a.sign > 0;
    const int total = TB * a.n;
    for (int e = tid; e < N; e += 256) {
        ltw[e] = tw[e];
        lhat[e] = hat[e];
    }
    for (int e = tid; e < a.n; e += 256) lw[e] = w[e];
    // The workgroup takes groups of TB transforms in turn (the tables above
    // are read once per workgroup); the next group's input is loaded into
    // registers while the current one is transformed.
    constexpr int KPT = (TB * 1024 + 255) / 256;   // staged values per thread (n <= 1024)
    const int n_groups = (a.nbatch + TB - 1) / TB;
    float2 pre[KPT];
    auto fetch = [&](int g) {
        const int gb0 = g * TB, gnb = min(TB, a.nbatch - gb0);
#pragma unroll
        for (int j = 0; j < KPT; ++j) {
            const int e = tid + 256 * j;
            pre[j] = make_float2(0.f, 0.f);
            if (e < total) {
                int t, i;
                if (a.n_fast_in) {
                    t = div_small(e, a.inv_n);
                    i = e - t * a.n;
                } else {
                    i = e / TB;
                    t = e - i * TB;
                }
                if (t < gnb) {
                    const int b = gb0 + t;
                    const int o = div_small(b, a.inv_inner), s = b - o * a.inner;
                    pre[j] = in[o * a.in_so + s * a.in_si + i * a.in_sn];
                }
            }
        }
    };
    if (blockIdx.x < n_groups) fetch(blockIdx.x);
    for (int grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const int b0 = grp * TB;
    const int nb = min(TB, a.nbatch - b0);
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const int e = tid + 256 * j;
        if (e < total) {
            int t, i;
            if (a.n_fast_in) {
                t = div_small(e, a.inv_n);
                i = e - t * a.n;
            } else {
                i = e / TB;
                t = e - i * TB;
            }
            stage[t * PS + i] = pre[j];
        }
    }
    __syncthreads();
    if (grp + static_cast<int>(gridDim.x) < n_groups) fetch(grp + gridDim.x);
    const int wave = tid >> 6, lane = tid & 63;
    float2* const A = lw + ((a.n + 1) & ~1) + wave * R * kWaveRow;   // this wavefront's rows
    for (int t = wave; t < nb; t += 4) {
        float2* X = stage + t * PS;
        // conj(x w), zero beyond n (x conjugated first for the inverse direction)
        float2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int idx = 64 * j + lane;
            float2 u = make_float2(0.f, 0.f);
            if (idx < a.n) {
                float2 x = X[idx];
                if (inv) x.y = -x.y;
                u = cmul(x, lw[idx]);
                u.y = -u.y;
            }
            v[j] = u;
        }
        // I: R-point transforms over a, twiddles wN^(l k1), rows k1
        idft_reg<R>(v);
#pragma unroll
        for (int k1 = 1; k1 < R; ++k1) {
            const float2 t1 = ltw[lane * k1];
            v[k1] = cmul(v[k1], make_float2(t1.x, -t1.y));
        }
        wave_lds_sync();   // the previous transform's last reads of the rows are done
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) A[k1 * kWaveRow + lane] = v[k1];
        wave_lds_sync();
        // I: first radix-8 pass over l2 (butterfly (k1, l1)), twiddles w64^(l1 m1)
        for (int b = lane; b < 8 * R; b += 64) {
            const int k1 = b >> 3, l1 = b & 7;
            float2* row = A + k1 * kWaveRow;
            float2 u[8];
#pragma unroll
            for (int l2 = 0; l2 < 8; ++l2) u[l2] = row[l1 + 8 * l2];
            dft_small<8>(u, +1);
#pragma unroll
            for (int m1 = 1; m1 < 8; ++m1) {
                const float2 t1 = ltw[R * l1 * m1];
                u[m1] = cmul(u[m1], make_float2(t1.x, -t1.y));
            }
#pragma unroll
            for (int m1 = 0; m1 < 8; ++m1) row[9 * m1 + l1] = u[m1];
        }
        wave_lds_sync();
        // I: second radix-8 pass over l1 (butterfly (k1, m1)) -> Y; Z = conj(Y) hat;
        // transposed pass over m2 back into the same eight places
        for (int b = lane; b < 8 * R; b += 64) {
            const int k1 = b >> 3, m1 = b & 7;
            float2* row = A + k1 * kWaveRow + 9 * m1;
            float2 u[8];
#pragma unroll
            for (int l1 = 0; l1 < 8; ++l1) u[l1] = row[l1];
            dft_small<8>(u, +1);
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2) u[m2] = cmul(make_float2(u[m2].x, -u[m2].y), lhat[k1 + R * (m1 + 8 * m2)]);
            dft_small<8>(u, +1);
#pragma unroll
            for (int l1 = 0; l1 < 8; ++l1) row[l1] = u[l1];
        }
        wave_lds_sync();
        // transposed pass over m1 (butterfly (k1, l1)), twiddles w64^(l1 m1) first
        for (int b = lane; b < 8 * R; b += 64) {
            const int k1 = b >> 3, l1 = b & 7;
            float2* row = A + k1 * kWaveRow;
            float2 u[8];
#pragma unroll
            for (int m1 = 0; m1 < 8; ++m1) u[m1] = row[9 * m1 + l1];
#pragma unroll
            for (int m1 = 1; m1 < 8; ++m1) {
                const float2 t1 = ltw[R * l1 * m1];
                u[m1] = cmul(u[m1], make_float2(t1.x, -t1.y));
            }
            dft_small<8>(u, +1);
#pragma unroll
            for (int l2 = 0; l2 < 8; ++l2) row[l1 + 8 * l2] = u[l2];
        }
        wave_lds_sync();
        // transposed pass over k1 (lane l): twiddles wN^(l k1), R-point sums -> c[64 a + l]
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) v[k1] = A[k1 * kWaveRow + lane];
#pragma unroll
        for (int k1 = 1; k1 < R; ++k1) {
            const float2 t1 = ltw[lane * k1];
            v[k1] = cmul(v[k1], make_float2(t1.x, -t1.y));
        }
        idft_reg<R>(v);
        // X = w c for k < n (conjugated for the inverse direction), in place of the input
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int idx = 64 * j + lane;
            if (idx < a.n) {
                float2 y = cmul(v[j], lw[idx]);
                if (inv) y.y = -y.y;
                X[idx] = y;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < total; e += 256) {
        int t, i;
        if (a.n_fast_out) {
            t = div_small(e, a.inv_n);
            i = e - t * a.n;
        } else {
            i = e / TB;
            t = e - i * TB;
        }
        if (t < nb) {
            const int b = b0 + t;
            const int o = div_small(b, a.inv_inner), s = b - o * a.inner;
            out[o * a.out_so + s * a.out_si + i * a.out_sn] = cscale(stage[t * PS + i], a.scale);
        }
    }
    __syncthreads();   // the staged transforms are stored before the next group is staged
    }
}

template <int R>
int launch_chirp_wave(const FftArgs& a, const float2* in, float2* out, const float2* tw, const float2* w,
                      const float2* hat, hipStream_t s, const char* what) {
    constexpr int TB = 4;   // one transform per wavefront: two workgroups per CU up to R = 16
    const size_t smem = (((static_cast<size_t>(TB) * (a.n | 1) + 1) & ~1ull) + 2ull * 64 * R +
                         ((static_cast<size_t>(a.n) + 1) & ~1ull) + 4ull * R * kWaveRow) * sizeof(float2);
    auto fn = fft_chirp_wave_kernel<R, TB>;
    int rc = set_lds_limit(reinterpret_cast<const void*>(fn), smem, what);
    if (rc) return rc;
    // as many workgroups as are resident at once, each taking groups of
    // transforms in turn
    const long long groups = (static_cast<long long>(a.nbatch) + TB - 1) / TB;
    rc = resident_grid(reinterpret_cast<const void*>(fn), smem, what, groups);
    if (rc <= 0) return -rc;
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(rc)), dim3(256), smem, s, in, out, tw, w, hat, a);
    return check_launch(what);
}

template <int R>
int launch_fft_wave(const FftArgs& a, const float2* in, float2* out, const float2* tw, hipStream_t s,
                    const char* what) {
    // sixteen transforms per workgroup of eight wavefronts: 128-byte runs on
    // the strided side (measured 10 % faster than eight transforms on four
    // wavefronts with 64-byte runs; sixteen on four wavefronts, half the
    // resident wavefronts, had run 15-20 % slower)
    constexpr int TB = 16, NW = 8;
    const size_t smem = static_cast<size_t>(TB) * (kWaveRow * R + 2) * sizeof(float2);
    auto fn = fft_wave_strided_kernel<R, TB, NW>;
    if (smem > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            static_cast<int>(smem)) != hipSuccess)
        return fail(PL_EDEVICE, "%s: LDS of %zu bytes refused", what, smem);
    const long long blocks = (static_cast<long long>(a.nbatch) + TB - 1) / TB;
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(64 * NW), smem, s, in, out, tw, a);
    return check_launch(what);
}

int set_lds_limit(const void* fn, size_t smem, const char* what) {
    if (smem > kMaxLds) return fail(PL_EUNSUPPORTED, "%s: LDS of %zu bytes exceeds the workgroup's", what, smem);
    if (smem > 65536 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem)) != hipSuccess)
        return fail(PL_EDEVICE, "%s: LDS of %zu bytes refused", what, smem);
    return PL_OK;
}

// Batched transforms of length f.n along a strided axis; the tables of f are
// at `tables` (device).
int run_fft(const float2* in, float2* out, const AxisFft& f, const char* tables, long long nbatch, int inner,
            long long in_so, long long in_si, long long in_sn, long long out_so, long long out_si,
            long long out_sn, int sign, float scale, hipStream_t s, const char* what) {
    FftArgs a{};
    a.n = f.n;
    a.m = f.m;
    a.nbatch = static_cast<int>(nbatch);
    a.inner = inner;
    a.per_wg = std::max(1, std::min(64, 2048 / f.m));
    a.ld = f.m + 1;
    a.sign = sign;
    a.n_fast_in = in_sn == 1;
    a.n_fast_out = out_sn == 1;
    a.in_so = in_so;
    a.in_si = in_si;
    a.in_sn = in_sn;
    a.out_so = out_so;
    a.out_si = out_si;
    a.out_sn = out_sn;
    a.scale = scale;
    a.inv_inner = 1.0f / inner;
    a.inv_n = 1.0f / f.n;
    a.inv_m = 1.0f / f.m;
    a.inv_pad = f.m > f.n ? 1.0f / (f.m - f.n) : 1.0f;
    a.rad = f.rad;
    if (nbatch <= 0) return PL_OK;
    if (nbatch > (1LL << 31) - 1) return fail(PL_EUNSUPPORTED, "%s: too many transforms", what);
    const float2* tw = reinterpret_cast<const float2*>(tables + f.off_tw);
    if (f.chirp && f.m % 64 == 0 && 2 * f.n <= f.m && nbatch + inner < (1LL << 21)) {
        // the wavefront chirp-z kernel (float-reciprocal index splits: exact
        // below 2^21 with its TB * n element loop)
        const float2* w = reinterpret_cast<const float2*>(tables + f.off_chirp);
        const float2* hat = reinterpret_cast<const float2*>(tables + f.off_hat);
        switch (f.m / 64) {
#define PL_CW(R) \
            case R: return launch_chirp_wave<R>(a, in, out, tw, w, hat, s, what);
            PL_CW(2) PL_CW(3) PL_CW(4) PL_CW(5) PL_CW(6) PL_CW(8) PL_CW(9) PL_CW(10) PL_CW(12) PL_CW(15) PL_CW(16)
            PL_CW(18) PL_CW(20) PL_CW(24) PL_CW(25) PL_CW(27) PL_CW(30) PL_CW(32)
#undef PL_CW
            default: break;
        }
    }
    if (f.chirp) {
        // the chirp kernel splits indices with float reciprocals (div_small):
        // exact while index + divisor < 2^22
        if (nbatch + inner >= (1LL << 22))
            return fail(PL_EUNSUPPORTED, "%s: %lld chirp-z transforms exceed the index range", what, nbatch);
        const size_t smem = 2ull * a.per_wg * a.ld * sizeof(float2);
        int rc = set_lds_limit(reinterpret_cast<const void*>(fft_chirp_strided_kernel), smem, what);
        if (rc) return rc;
        const long long blocks = (nbatch + a.per_wg - 1) / a.per_wg;
        hipLaunchKernelGGL(fft_chirp_strided_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, in, out,
                           tw, reinterpret_cast<const float2*>(tables + f.off_chirp),
                           reinterpret_cast<const float2*>(tables + f.off_hat), a);
        return check_launch(what);
    }
    // the wavefront kernel splits batch indices with a float reciprocal (exact
    // below 2^22)
    if (f.n % 64 == 0 && nbatch + inner < (1LL << 21)) {
        switch (f.n / 64) {
            case 2: return launch_fft_wave<2>(a, in, out, tw, s, what);
            case 3: return launch_fft_wave<3>(a, in, out, tw, s, what);
            case 4: return launch_fft_wave<4>(a, in, out, tw, s, what);
            case 5: return launch_fft_wave<5>(a, in, out, tw, s, what);
            case 6: return launch_fft_wave<6>(a, in, out, tw, s, what);
            case 8: return launch_fft_wave<8>(a, in, out, tw, s, what);
            default: break;
        }
    }
    const size_t smem = 2ull * a.per_wg * a.ld * sizeof(float2);
    int rc = set_lds_limit(reinterpret_cast<const void*>(fft_strided_kernel), smem, what);
    if (rc) return rc;
    const long long blocks = (nbatch + a.per_wg - 1) / a.per_wg;
    hipLaunchKernelGGL(fft_strided_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), smem, s, in, out,
                       tw, a);
    return check_launch(what);
}

}  // namespace

int launch_plan_tables(const HybridPlan& p, const DeviceTables& dt, char* ws, hipStream_t s) {
    PlanTablesArgs a{};
    a.n_ch = p.n_ch;
    a.n_z = p.n_z;
    a.n_f = p.n_f;
    a.n_l = p.n_l;
    a.n_fine = p.n_fine;
    a.interp = p.interp;
    a.n_gl = p.n_gl;
    a.block = p.block;
    a.ref_mode = p.ref_mode;
    a.du = p.du;
    a.h = p.h;
    a.beta = p.beta;
    a.gx0 = p.x0;
    a.gx1 = p.x0 + (p.nx - 1) * p.dx;
    a.gy0 = p.y0;
    a.gy1 = p.y0 + (p.ny - 1) * p.dy;
    for (int b = 0; b < kMaxBlocks; ++b) a.kref[b] = p.kref[b];
    for (int q = 0; q < kMaxGL; ++q) {
        a.glx[q] = p.gl_x[q];
        a.glw[q] = p.gl_w[q];
    }
    a.scan_step = p.scan_step;
    const long long total = static_cast<long long>(p.n_ch) + p.n_z + p.n_fine + p.n_l +
                            static_cast<long long>(p.n_z) * p.n_f;
    const int blocks = static_cast<int>(std::min<long long>((total + 255) / 256, 4096));
    hipLaunchKernelGGL(plan_tables_kernel, dim3(blocks), dim3(256), 0, s, a, dt.chan, dt.k,
                       reinterpret_cast<double*>(ws + p.off_llo), reinterpret_cast<double*>(ws + p.off_lref),
                       reinterpret_cast<float2*>(ws + p.off_tw_fine), reinterpret_cast<float*>(ws + p.off_deap),
                       reinterpret_cast<double*>(ws + p.off_kp), reinterpret_cast<float*>(ws + p.off_wk),
                       reinterpret_cast<double*>(ws + p.off_krz));
    int rc = check_launch("plan tables");
    if (!rc) rc = launch_axis_fft_tables(p.zfft, ws + p.off_zfft, s);
    return rc ? rc : launch_tile_tables(p, dt, ws, s);
}

int launch_axis_fft_tables(const AxisFft& f, char* tables, hipStream_t s) {
    const int total = f.m + (f.chirp ? f.n + f.m : 0);
    hipLaunchKernelGGL(axis_fft_tables_kernel, dim3((total + 255) / 256), dim3(256), 0, s, f.n, f.m, f.chirp ? 1 : 0,
                       reinterpret_cast<float2*>(tables + f.off_tw), reinterpret_cast<float2*>(tables + f.off_chirp),
                       reinterpret_cast<float2*>(tables + f.off_pad));
    int rc = check_launch("transform tables");
    if (rc || !f.chirp) return rc;
    // hat = FFT_m(pad) / m: one smooth transform of length m
    AxisFft g = f;
    g.n = f.m;
    g.chirp = false;
    return run_fft(reinterpret_cast<const float2*>(tables + f.off_pad), reinterpret_cast<float2*>(tables + f.off_hat), g,
                   tables, 1, 1, 0, 0, 1, 0, 0, 1, -1, 1.0f / f.m, s, "transform tables (chirp filter)");
}

// s[c][m][f] -> S[c][kz][f]: forward transform over m (stride n_f).
int launch_scan_fft(const pl_geometry* g, const float2* echo, float2* spec, const AxisFft& f, const char* tables,
                    hipStream_t s) {
    const long long nf = g->n_freq, nz = g->n_scan;
    return run_fft(echo, spec, f, tables, static_cast<long long>(g->n_ch) * nf, g->n_freq, nz * nf, 1, nf, nz * nf, 1,
                   nf, -1, 1.0f, s, "scan fft");
}

// G[p][kz] -> g[z][p]: inverse transform over k_z with 1/n_z.
int launch_kz_ifft(const HybridPlan& p, const float2* G, float2* image, const char* tables, hipStream_t s) {
    const long long npix = static_cast<long long>(p.nx) * p.ny;
    return run_fft(G, image, p.zfft, tables, npix, 1, p.n_z, 0, 1, 1, 0, npix, +1, 1.0f / p.n_z, s, "kz ifft");
}

// g[z][p] -> G~[p][kz]: adjoint of launch_kz_ifft (forward transform over z
// with 1/n_z).
int launch_kz_fft_adjoint(const HybridPlan& p, const float2* image, float2* Gt, const char* tables, hipStream_t s) {
    const long long npix = static_cast<long long>(p.nx) * p.ny;
    return run_fft(image, Gt, p.zfft, tables, npix, 1, 1, 0, npix, p.n_z, 0, 1, -1, 1.0f / p.n_z, s,
                   "kz fft (adjoint)");
}

// S~[c][kz][f] -> s~[c][m][f]: adjoint of launch_scan_fft (unnormalised
// inverse transform over kz).
int launch_scan_fft_adjoint(const pl_geometry* g, const float2* St, float2* echo, const AxisFft& f,
                            const char* tables, hipStream_t s) {
    const long long nf = g->n_freq, nz = g->n_scan;
    return run_fft(St, echo, f, tables, static_cast<long long>(g->n_ch) * nf, g->n_freq, nz * nf, 1, nf, nz * nf, 1,
                   nf, +1, 1.0f, s, "scan fft (adjoint)");
}

}  // namespace pl
