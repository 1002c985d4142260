// Goldstein adaptive power-spectrum filter of the wrapped phase and the
// transfer of cycle counts back to the original phase (the optional
// preprocessing of Section II-D).
//
// The filter works on unit phasors (0 at invalid pixels and outside the
// image) in N x N patches on a grid of step S = N/2 whose first patch starts
// S rows above and S columns left of the image, so every pixel lies in four
// patches.  Per patch: the 2-D DFT Z, B = circular (2h+1)^2 mean of |Z|,
// Z * (B / max B)^alpha, the inverse DFT, tapered by w(r) w(c) with
// w(i) = 1 - |2i + 1 - N| / N.  The filtered phase is the argument of the
// sum of the four tapered patch outputs at each valid pixel.
//
//   k_gs_patch   one wave handles 64/N patches, N lanes per patch.  Lane k
//                loads column k of its patch straight into registers, so the
//                first 1-D DFT (over rows) needs no shuffle; one LDS
//                transpose turns columns into rows for the second.  The
//                spectrum stays in registers (lane = row u, register =
//                bit-reversed column v) for the smoothing: neighbours in v
//                are other registers, neighbours in u are lane shuffles.
//                The inverse runs the other way round (one more transpose)
//                and ends with lane k holding column k, so each output row
//                is written as one coalesced segment.  Each patch writes its
//                four S x S quadrants into four pixel-indexed planes (one
//                per quadrant position), so every pixel is written exactly
//                once per plane and no atomics are needed.
//   k_gs_combine sums the four planes per pixel in a fixed order (the
//                result does not depend on the schedule) and takes atan2.
//   k_gs_transfer  the cycle counts of the filtered phase moved onto the
//                original phase: K = K_f + k, k the integer that puts
//                psi + 2 pi K within (-pi, pi] of psi_f + 2 pi K_f.
//
// Radix-2 transforms in registers: decimation in frequency (natural order in,
// bit-reversed out) forward and decimation in time (bit-reversed in, natural
// out) inverse, so no reordering pass is ever made; the bit reversal is
// absorbed into the compile-time register and LDS indices.  Twiddles are
// compile-time constants.
#include "ww_internal.h"

namespace ww {

namespace {

// sin and cos by their Taylor series at compile time (|x| <= pi here; 30
// terms leave an error far below float precision).
constexpr double cx_sin(double x) {
    double t = x, s = x;
    for (int k = 1; k < 30; ++k) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}

constexpr double cx_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 30; ++k) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}

template <int N>
struct Twiddles {
    float c[N / 2];
    float s[N / 2];
};

// W_N^k = exp(-2 pi i k / N) = c[k] - i s[k], k < N/2
template <int N>
constexpr Twiddles<N> make_twiddles() {
    Twiddles<N> t{};
    for (int k = 0; k < N / 2; ++k) {
        const double a = 2.0 * PI_D * (double)k / (double)N;
        t.c[k] = (float)cx_cos(a);
        t.s[k] = (float)cx_sin(a);
    }
    return t;
}

template <int N>
constexpr int ilog2() {
    int l = 0;
    while ((1 << l) < N) ++l;
    return l;
}

template <int N>
constexpr int bitrev(int j) {
    int r = 0;
    for (int b = 0; b < ilog2<N>(); ++b)
        if (j & (1 << b)) r |= 1 << (ilog2<N>() - 1 - b);
    return r;
}

// Forward DFT, decimation in frequency: x natural in, X[bitrev(j)] in
// register j out.  Unnormalised, exponent -2 pi i.
template <int N>
__device__ __forceinline__ void dft_dif(float (&re)[N], float (&im)[N]) {
    constexpr Twiddles<N> tw = make_twiddles<N>();
#pragma unroll
    for (int h = N / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int b0 = 0; b0 < N; b0 += 2 * h) {
#pragma unroll
            for (int t = 0; t < h; ++t) {
                const int i = b0 + t, j = i + h;
                const float ar = re[i], ai = im[i], br = re[j], bi = im[j];
                re[i] = ar + br;
                im[i] = ai + bi;
                const float dr = ar - br, di = ai - bi;
                const int k = t * (N / (2 * h));
                if (k == 0) {  // W = 1
                    re[j] = dr;
                    im[j] = di;
                } else if (4 * k == N) {  // W = -i
                    re[j] = di;
                    im[j] = -dr;
                } else {
                    const float c = tw.c[k], s = tw.s[k];
                    // (dr + i di)(c - i s)
                    re[j] = dr * c + di * s;
                    im[j] = di * c - dr * s;
                }
            }
        }
    }
}

// Inverse DFT, decimation in time: X[bitrev(j)] in register j in, x natural
// out.  Unnormalised, exponent +2 pi i.
template <int N>
__device__ __forceinline__ void idft_dit(float (&re)[N], float (&im)[N]) {
    constexpr Twiddles<N> tw = make_twiddles<N>();
#pragma unroll
    for (int h = 1; h < N; h <<= 1) {
#pragma unroll
        for (int b0 = 0; b0 < N; b0 += 2 * h) {
#pragma unroll
            for (int t = 0; t < h; ++t) {
                const int i = b0 + t, j = i + h;
                const int k = t * (N / (2 * h));
                float tr, ti;
                if (k == 0) {  // W = 1
                    tr = re[j];
                    ti = im[j];
                } else if (4 * k == N) {  // W = +i
                    tr = -im[j];
                    ti = re[j];
                } else {
                    const float c = tw.c[k], s = tw.s[k];
                    // x_j (c + i s)
                    tr = re[j] * c - im[j] * s;
                    ti = im[j] * c + re[j] * s;
                }
                const float ar = re[i], ai = im[i];
                re[i] = ar + tr;
                im[i] = ai + ti;
                re[j] = ar - tr;
                im[j] = ai - ti;
            }
        }
    }
}

template <int N>
constexpr float taper(int i) {
    const int d = 2 * i + 1 - N;
    return (float)(N - (d < 0 ? -d : d)) / (float)N;
}

}  // namespace

constexpr int GS_PLANES = 4;

template <int N, int SH>
__global__ __launch_bounds__(64, (N == 32 ? 3 : 1)) void k_gs_patch(const float *__restrict__ psi,
                                                 const uint8_t *__restrict__ valid, int m, int n,
                                                 int PJ, int64_t npatch, float alpha,
                                                 float2 *__restrict__ planes, int64_t pstride) {
    constexpr int G = 64 / N, S = N / 2, LP = N + 1;
    __shared__ float tre[G * N * LP];
    __shared__ float tim[G * N * LP];
    const int lane = threadIdx.x, g = lane / N, k = lane % N;
    const int64_t p = (int64_t)blockIdx.x * G + g;
    const bool live = p < npatch;
    const int pi = live ? (int)(p / PJ) : 0, pj = live ? (int)(p % PJ) : 0;
    const int r0 = pi * S - S, c0 = pj * S - S;
    const int c = c0 + k;
    const bool cin = live && c >= 0 && c < n;

    float re[N], im[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const int r = r0 + a;
        float x = 0.f;
        bool on = cin && r >= 0 && r < m;
        if (on) {
            const int64_t idx = (int64_t)r * n + c;
            x = psi[idx];
            if (valid) on = valid[idx] != 0;
        }
        // exp(i x) through sinpi/cospi of x / pi: a short reduction for any x
        float sv, cv;
        sincospif(x * (float)(1.0 / PI_D), &sv, &cv);
        re[a] = on ? cv : 0.f;
        im[a] = on ? sv : 0.f;
    }
    // DFT over rows: lane k holds column k, register j = row frequency bitrev(j)
    dft_dif<N>(re, im);
    float *Tr = tre + g * N * LP, *Ti = tim + g * N * LP;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        Tr[bitrev<N>(j) * LP + k] = re[j];
        Ti[bitrev<N>(j) * LP + k] = im[j];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < N; ++b) {
        re[b] = Tr[k * LP + b];
        im[b] = Ti[k * LP + b];
    }
    // DFT over columns: lane u = k holds spectrum row u, register j = Z[u][bitrev(j)]
    dft_dif<N>(re, im);

    // B = circular (2 SH + 1)^2 mean of |Z|, up to the common factor
    float R[N];
    {
        float A[N];
#pragma unroll
        for (int j = 0; j < N; ++j) A[j] = __builtin_amdgcn_sqrtf(re[j] * re[j] + im[j] * im[j]);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            float s = 0.f;
#pragma unroll
            for (int dv = -SH; dv <= SH; ++dv) s += A[bitrev<N>((bitrev<N>(j) + dv + N) % N)];
            R[j] = s;
        }
    }
    const int base = g * N;
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        float s = R[j];
#pragma unroll
        for (int du = 1; du <= SH; ++du) {
            s += __shfl(R[j], base + ((k + du) & (N - 1)), 64);
            s += __shfl(R[j], base + ((k - du + N) & (N - 1)), 64);
        }
        R[j] = s;
        mx = fmaxf(mx, s);
    }
#pragma unroll
    for (int off = N / 2; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    // H = (B / max B)^alpha by the hardware base-2 logarithm and exponential
    // (B = 0 gives log2 = -inf and H = 0); alpha = 0 leaves Z unchanged
    if (alpha != 0.f) {
        const float inv = mx > 0.f ? 1.f / mx : 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const float H = __builtin_amdgcn_exp2f(alpha * __builtin_amdgcn_logf(R[j] * inv));
            re[j] *= H;
            im[j] *= H;
        }
    }

    // inverse over columns: register j (= bitrev column) in, natural column out
    idft_dit<N>(re, im);
    __syncthreads();  // every lane has read the first transpose
#pragma unroll
    for (int b = 0; b < N; ++b) {
        Tr[k * LP + b] = re[b];
        Ti[k * LP + b] = im[b];
    }
    __syncthreads();
    // lane k = column b; rows in bit-reversed order for the inverse over rows
#pragma unroll
    for (int j = 0; j < N; ++j) {
        re[j] = Tr[bitrev<N>(j) * LP + k];
        im[j] = Ti[bitrev<N>(j) * LP + k];
    }
    idft_dit<N>(re, im);

    if (!cin) return;
    const float wk = (float)(N - abs(2 * k + 1 - N)) / (float)N * (1.f / (float)(N * N));
    float2 *qcol = planes + (k >= S ? 1 : 0) * pstride;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const int r = r0 + a;
        if (r < 0 || r >= m) continue;
        const float w = taper<N>(a) * wk;
        float2 *q = qcol + (a >= S ? 2 : 0) * pstride;
        q[(int64_t)r * n + c] = make_float2(re[a] * w, im[a] * w);
    }
}

__global__ __launch_bounds__(256) void k_gs_combine(const float2 *__restrict__ planes,
                                                    int64_t pstride, const float *__restrict__ psi,
                                                    const uint8_t *__restrict__ valid, int64_t total,
                                                    float *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (valid && !valid[i]) {
            out[i] = psi[i];
            continue;
        }
        const float2 a = planes[i], b = planes[i + pstride], c = planes[i + 2 * pstride],
                     d = planes[i + 3 * pstride];
        const float x = ((a.x + b.x) + c.x) + d.x, y = ((a.y + b.y) + c.y) + d.y;
        out[i] = atan2f(y, x);
    }
}

// Shift that gives the reference pixel K = 0 after the transfer (0 when
// there is no reference).
__global__ void k_gs_ref_shift(const float *__restrict__ psi, const uint8_t *__restrict__ valid,
                               const float *__restrict__ psi_f, const int32_t *__restrict__ K_f,
                               int64_t total, int64_t ref_host, const long long *ref_dev,
                               int32_t *shift) {
#pragma clang fp contract(off)
    const int64_t ref = ref_dev ? (int64_t)*ref_dev : ref_host;
    int32_t s = 0;
    if (ref >= 0 && ref < total) {
        s = K_f[ref];
        if (!valid || valid[ref]) {
            const double x = (double)psi[ref] - (double)psi_f[ref];
            s -= (x > PI_D) - (x <= -PI_D);
        }
    }
    *shift = s;
}

__global__ __launch_bounds__(256) void k_gs_transfer(
    const float *__restrict__ psi, const uint8_t *__restrict__ valid,
    const float *__restrict__ psi_f, const int32_t *K_f, int64_t total, const int32_t *shift,
    float nodata, int32_t *K, float *__restrict__ phi) {
#pragma clang fp contract(off)
    const int32_t sh = *shift;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t kf = K_f[i];
        if (valid && !valid[i]) {
            K[i] = kf - sh;
            phi[i] = nodata;
            continue;
        }
        const double p = (double)psi[i];
        const double x = p - (double)psi_f[i];
        const int32_t kv = kf - ((x > PI_D) - (x <= -PI_D)) - sh;
        K[i] = kv;
        phi[i] = (float)(p + TWO_PI_D * (double)kv);
    }
}

ww_status goldstein_impl(const float *psi, const uint8_t *valid, int m, int n,
                         const ww_filter_params &fp, float *out, hipStream_t stream) {
    const int64_t total = (int64_t)m * n;
    if (total == 0) return WW_OK;
    const int N = fp.patch, S = N / 2, SH = fp.smooth / 2;
    float2 *planes = nullptr;
    WW_TRY(scratch(SLOT_GS_PLANES, (size_t)GS_PLANES * (size_t)total * sizeof(float2),
                   (void **)&planes));
    const int PI = (m + S - 1) / S + 1, PJ = (n + S - 1) / S + 1;
    const int64_t npatch = (int64_t)PI * PJ;
    const int G = 64 / N;
    const int64_t nblk = (npatch + G - 1) / G;
    if (nblk >= ((int64_t)1 << 31)) return fail(WW_E_INVALID_ARG, "image too large for the filter");
#define WW_GS(NN, HH)                                                                           \
    hipLaunchKernelGGL((k_gs_patch<NN, HH>), dim3((unsigned)nblk), dim3(64), 0, stream, psi,    \
                       valid, m, n, PJ, npatch, fp.alpha, planes, total)
#define WW_GS_H(NN)                   \
    switch (SH) {                     \
        case 0: WW_GS(NN, 0); break;  \
        case 1: WW_GS(NN, 1); break;  \
        default: WW_GS(NN, 2); break; \
    }
    switch (N) {
        case 16: WW_GS_H(16) break;
        case 32: WW_GS_H(32) break;
        default: WW_GS_H(64) break;
    }
#undef WW_GS_H
#undef WW_GS
    WW_LAUNCH_CHECK();
    const int64_t cblk = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gs_combine, dim3((unsigned)cblk), dim3(256), 0, stream, planes, total,
                       psi, valid, total, out);
    WW_LAUNCH_CHECK();
    return WW_OK;
}

ww_status transfer_impl(const float *psi, const uint8_t *valid, const float *psi_f,
                        const int32_t *K_f, int m, int n, int64_t ref_host,
                        const long long *ref_dev, float nodata, int32_t *K, float *phi,
                        hipStream_t stream) {
    const int64_t total = (int64_t)m * n;
    if (total == 0) return WW_OK;
    int32_t *shift = nullptr;
    WW_TRY(scratch(SLOT_GS_SHIFT, 256, (void **)&shift));
    hipLaunchKernelGGL(k_gs_ref_shift, dim3(1), dim3(1), 0, stream, psi, valid, psi_f, K_f, total,
                       ref_host, ref_dev, shift);
    WW_LAUNCH_CHECK();
    const int64_t blk = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gs_transfer, dim3((unsigned)blk), dim3(256), 0, stream, psi, valid, psi_f,
                       K_f, total, shift, nodata, K, phi);
    WW_LAUNCH_CHECK();
    return WW_OK;
}

}  // namespace ww
