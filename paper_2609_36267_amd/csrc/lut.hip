// Integer cost table of Section II-B (eqs. 4-7), built in FP64 on the GPU.
//
// Discretisation (identical on every implementation of the table):
//   eta_i   = -pi + (i + 1/2) deta, deta = 2pi/n_eta              (phase noise)
//   gamma_k : composite Gauss-Legendre rule on [0,1] (n_gpanel panels of
//             n_gnode nodes) for the true-coherence integral of eq. 5
//   f~_c    = sum_k W_k f_eta(eta_i|gamma_k) f_T(gh_c|gamma_k), unit mass
//   p_c(s)  = deta^2 sum_i f~_c(i+s) f~_c(i), s = -(n_eta-1)..(n_eta-1),
//             spread uniformly over the cell [(s-1/2)deta, (s+1/2)deta]
//   q0, q+  : eq. 6 from the left/right cumulative sums of p_c, linear inside
//             a cell; q0 from the right tail when alpha <= 0 (small tails
//             never come from 1 - G)
//   sigma_c = sqrt(sum_i eta_i^2 f_eta(eta_i|gh_c) deta)
//   P_j     = sum_k om_k q_j(ah_b + span sigma_c (2k/(n_aquad-1) - 1)),
//             om_k = normalised exp(-u_k^2/2)                         (eq. 7)
//   T[c][b] = min(32767, floor(100 max(0, -log(P+/P0)))), 32767 if P+ = 0.
//
// f_eta is Lee et al.'s multilook phase density.  With beta = gamma cos eta,
// f_eta = (1-g^2)^L/(2pi(2L+1)) 2F1(2,2L;L+3/2;(1+beta)/2) is a sum of
// positive terms for beta <= 0; for beta > 0 the series is taken at -beta and
// the odd term of the published two-term form is added twice, which again
// adds positive quantities.  The published two-term form itself loses every
// digit in the tails and is not used.
//
// The work is tiny (a few hundred MFLOP per table) and cached per L, so the
// kernels favour plainness: one thread per output, sequential inner sums,
// deterministic reduction orders.
#pragma clang fp contract(off)

#include <cmath>

#include "ww_internal.h"

namespace ww {

namespace {

__device__ double log_1m_sq(double x) { return log1p(-x) + log1p(x); }

// 2F1(2, 2L; L+3/2; z), 0 <= z <= 1/2, all terms positive.
__device__ double hyp_series(int L, double z) {
    double sum = 0.0, term = 1.0;
    const double a = 2.0, b = 2.0 * L, c = L + 1.5;
    for (int k = 0; k < 200000; ++k) {
        sum += term;
        double ratio = (a + k) * (b + k) / ((c + k) * (k + 1.0)) * z;
        term *= ratio;
        if (ratio < 1.0 && term < sum * 8.673617379884035e-19) break;
    }
    return sum;
}

__device__ double f_eta_dev(double eta, double g, int L) {
    const double beta = g * cos(eta);
    const double lg = log_1m_sq(g);
    const double front = exp((double)L * lg) / (2.0 * PI_D * (2.0 * L + 1.0));
    double val = front * hyp_series(L, 0.5 * (1.0 - fabs(beta)));
    if (beta > 0.0) {
        const double lb = log_1m_sq(beta);
        const double odd = exp(lgamma(L + 0.5) - lgamma((double)L) + (double)L * (lg - lb) - 0.5 * lb) *
                           beta / (2.0 * sqrt(PI_D));
        val += 2.0 * odd;
    }
    return val;
}

// Touzi et al.'s density of the sample coherence gh given gamma (L >= 2).
__device__ double touzi_dev(double gh, double g, int L) {
    if (gh <= 0.0 || gh >= 1.0) return 0.0;
    const double x = g * g * gh * gh;
    const double lpre = log(2.0 * (L - 1)) + (double)L * log_1m_sq(g) + log(gh) +
                        (double)(L - 2) * log_1m_sq(gh) + (double)(1 - 2 * L) * log1p(-x);
    double poly = 0.0, binom = 1.0, xk = 1.0;
    for (int k = 0; k < L; ++k) {
        poly += binom * binom * xk;
        binom = binom * (double)(L - 1 - k) / (double)(k + 1);
        xk *= x;
    }
    return exp(lpre) * poly;
}

}  // namespace

// Gauss-Legendre rule on [-1,1] by Newton iteration on the three-term
// recurrence, mapped onto n_gpanel equal panels of [0,1].
__global__ void k_gl_rule(int Q, int P, double *gx, double *gw) {
    const int q = threadIdx.x;
    if (q >= Q) return;
    double x = cos(PI_D * (q + 0.75) / (Q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 64; ++it) {
        double pm1 = 1.0, p = x;
        for (int k = 2; k <= Q; ++k) {
            double pn = ((2.0 * k - 1.0) * x * p - (k - 1.0) * pm1) / (double)k;
            pm1 = p;
            p = pn;
        }
        if (Q == 1) { p = x; pm1 = 1.0; }
        dp = Q * (x * p - pm1) / (x * x - 1.0);
        double step = p / dp;
        x -= step;
        if (fabs(step) < 1e-16) break;
    }
    {
        double pm1 = 1.0, p = x;
        for (int k = 2; k <= Q; ++k) {
            double pn = ((2.0 * k - 1.0) * x * p - (k - 1.0) * pm1) / (double)k;
            pm1 = p;
            p = pn;
        }
        if (Q == 1) { p = x; pm1 = 1.0; }
        dp = Q * (x * p - pm1) / (x * x - 1.0);
    }
    const double node = -x, weight = 2.0 / ((1.0 - x * x) * dp * dp);
    for (int pa = 0; pa < P; ++pa) {
        gx[pa * Q + q] = (pa + 0.5 * (1.0 + node)) / P;
        gw[pa * Q + q] = weight / (2.0 * P);
    }
}

// fe[k*H + i] = f_eta(eta_i | gamma_k), i < H = n_eta/2 (f_eta is even in eta).
__global__ void k_feta_table(int L, int N, int NQ, const double *gx, double *fe) {
    const int H = N / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NQ * H) return;
    const int k = (int)(t / H), i = (int)(t % H);
    const double deta = TWO_PI_D / N;
    fe[t] = f_eta_dev(-PI_D + (i + 0.5) * deta, gx[k], L);
}

// tw[c*NQ + k] = W_k f_T(gh_c | gamma_k)
__global__ void k_touzi_weights(int L, int NG, int NQ, const double *gx, const double *gw,
                                double *tw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NG * NQ) return;
    const int c = (int)(t / NQ), k = (int)(t % NQ);
    tw[t] = gw[k] * touzi_dev((c + 0.5) / NG, gx[k], L);
}

// half-range f~ before normalisation: ft[c*H + i] = sum_k tw[c][k] fe[k][i]
__global__ void k_ftilde(int NG, int NQ, int H, const double *tw, const double *fe, double *ft) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NG * H) return;
    const int c = (int)(t / H), i = (int)(t % H);
    double acc = 0.0;
    for (int k = 0; k < NQ; ++k) acc += tw[(int64_t)c * NQ + k] * fe[(int64_t)k * H + i];
    ft[t] = acc;
}

// Unit mass on (-pi, pi] (both halves), then expand to the full eta range.
__global__ void k_ftilde_normalise(int NG, int N, const double *half, double *full) {
    const int c = blockIdx.x;
    const int H = N / 2;
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < H; i += blockDim.x) s += half[(int64_t)c * H + i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double mass = 2.0 * part[0] * (TWO_PI_D / N);
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        double v = half[(int64_t)c * H + i] / mass;
        full[(int64_t)c * N + i] = v;
        full[(int64_t)c * N + (N - 1 - i)] = v;
    }
}

// pm[c*(2N-1) + s + N-1] = deta^2 sum_i f~(i+s) f~(i), symmetric in s.
__global__ void k_edge_mass(int NG, int N, const double *ft, double *pm) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NG * N) return;
    const int c = (int)(t / N), s = (int)(t % N);  // s = 0..N-1
    const double *f = ft + (int64_t)c * N;
    double acc = 0.0;
    for (int i = 0; i + s < N; ++i) acc += f[i + s] * f[i];
    const double deta = TWO_PI_D / N;
    const double v = acc * deta * deta;
    double *p = pm + (int64_t)c * (2 * N - 1);
    p[N - 1 + s] = v;
    p[N - 1 - s] = v;
}

// Left/right cumulative sums at the cell edges k = -(N-1)..N, stored at k+N-1:
// CL = mass below edge k, CR = mass at or above edge k.  One thread per row.
__global__ void k_cumsums(int NG, int N, const double *pm, double *CL, double *CR) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NG) return;
    const double *p = pm + (int64_t)c * (2 * N - 1);
    double *L = CL + (int64_t)c * 2 * N, *R = CR + (int64_t)c * 2 * N;
    double acc = 0.0;
    L[0] = 0.0;
    for (int e = 1; e < 2 * N; ++e) {
        acc += p[e - 1];
        L[e] = acc;
    }
    acc = 0.0;
    R[2 * N - 1] = 0.0;
    for (int e = 2 * N - 2; e >= 0; --e) {
        acc += p[e];
        R[e] = acc;
    }
}

// sigma_alpha of each coherence bin: std of f_eta at gamma = gh_c.
__global__ void k_sigma(int L, int NG, int N, double *sig) {
    const int c = blockIdx.x;
    const double gh = (c + 0.5) / NG, deta = TWO_PI_D / N;
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double eta = -PI_D + (i + 0.5) * deta;
        s += eta * eta * f_eta_dev(eta, gh, L) * deta;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sig[c] = sqrt(part[0]);
}

// Normalised Gaussian slope weights (one block).
__global__ void k_slope_weights(int NA, double span, double *om) {
    __shared__ double part[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < NA; k += blockDim.x) {
        double u = span * (2.0 * k / (NA - 1) - 1.0);
        double w = exp(-0.5 * u * u);
        om[k] = w;
        s += w;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double tot = part[0];
    __syncthreads();
    for (int k = threadIdx.x; k < NA; k += blockDim.x) om[k] /= tot;
}

namespace {
struct Cdf {
    const double *p, *L, *R;
    int N;
    double deta;
    __device__ double below(double x) const {
        double u = x / deta + 0.5;
        double fk = floor(u);
        if (fk < -(N - 1)) return 0.0;
        if (fk > N - 1) return L[2 * N - 1];
        int k = (int)fk;
        return L[k + N - 1] + (u - fk) * p[k + N - 1];
    }
    __device__ double above(double x) const {
        double u = x / deta + 0.5;
        double fk = floor(u);
        if (fk < -(N - 1)) return R[0];
        if (fk > N - 1) return 0.0;
        int k = (int)fk;
        return R[k + N] + (1.0 - (u - fk)) * p[k + N - 1];
    }
};
}  // namespace

__global__ void k_table(int NG, int NAl, int N, int NA, double span, const double *pm,
                        const double *CL, const double *CR, const double *sig, const double *om,
                        int16_t *T) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)NG * NAl) return;
    const int c = (int)(t / NAl), b = (int)(t % NAl);
    Cdf cdf;
    cdf.p = pm + (int64_t)c * (2 * N - 1);
    cdf.L = CL + (int64_t)c * 2 * N;
    cdf.R = CR + (int64_t)c * 2 * N;
    cdf.N = N;
    cdf.deta = TWO_PI_D / N;
    const double ah = -PI_D + (b + 0.5) * TWO_PI_D / NAl;
    const double sg = sig[c];
    double P0 = 0.0, Pp = 0.0;
    for (int k = 0; k < NA; ++k) {
        const double a = ah + span * sg * (2.0 * k / (NA - 1) - 1.0);
        double q0;
        if (a <= 0.0) q0 = cdf.above(-PI_D - a) - cdf.above(PI_D - a);
        else q0 = cdf.below(PI_D - a) - cdf.below(-PI_D - a);
        const double qp = cdf.above(PI_D - a);
        P0 += om[k] * q0;
        Pp += om[k] * qp;
    }
    int16_t out;
    if (!(Pp > 0.0)) {
        out = 32767;
    } else {
        double cst = -log(Pp / P0);
        if (cst < 0.0) cst = 0.0;
        double v = floor(100.0 * cst);
        out = v >= 32767.0 ? (int16_t)32767 : (int16_t)v;
    }
    T[t] = out;
}

ww_status build_lut_impl(int looks, const ww_lut_params &p, int16_t *lut_dev, hipStream_t st) {
    const int N = p.n_eta, H = N / 2, NG = p.n_gamma, NAl = p.n_alpha, NA = p.n_aquad;
    const int NQ = p.n_gpanel * p.n_gnode;
    size_t off = 0;
    auto carve = [&](size_t count) {
        size_t o = off;
        off += ((count * sizeof(double) + 255) / 256) * 256;
        return o;
    };
    const size_t o_gx = carve(NQ), o_gw = carve(NQ), o_fe = carve((size_t)NQ * H),
                 o_tw = carve((size_t)NG * NQ), o_half = carve((size_t)NG * H),
                 o_ft = carve((size_t)NG * N), o_pm = carve((size_t)NG * (2 * N - 1)),
                 o_cl = carve((size_t)NG * 2 * N), o_cr = carve((size_t)NG * 2 * N),
                 o_sig = carve(NG), o_om = carve(NA);
    char *base = nullptr;
    WW_TRY(scratch(SLOT_LUT_WORK, off, (void **)&base));
    double *gx = (double *)(base + o_gx), *gw = (double *)(base + o_gw),
           *fe = (double *)(base + o_fe), *tw = (double *)(base + o_tw),
           *half = (double *)(base + o_half), *ft = (double *)(base + o_ft),
           *pm = (double *)(base + o_pm), *cl = (double *)(base + o_cl),
           *cr = (double *)(base + o_cr), *sig = (double *)(base + o_sig),
           *om = (double *)(base + o_om);
    const int TB = 256;
    hipLaunchKernelGGL(k_gl_rule, dim3(1), dim3(64), 0, st, p.n_gnode, p.n_gpanel, gx, gw);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_feta_table, dim3(ceil_div((int64_t)NQ * H, TB)), dim3(TB), 0, st, looks,
                       N, NQ, gx, fe);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_touzi_weights, dim3(ceil_div((int64_t)NG * NQ, TB)), dim3(TB), 0, st,
                       looks, NG, NQ, gx, gw, tw);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ftilde, dim3(ceil_div((int64_t)NG * H, TB)), dim3(TB), 0, st, NG, NQ, H,
                       tw, fe, half);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ftilde_normalise, dim3(NG), dim3(256), 0, st, NG, N, half, ft);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_edge_mass, dim3(ceil_div((int64_t)NG * N, TB)), dim3(TB), 0, st, NG, N,
                       ft, pm);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cumsums, dim3(ceil_div(NG, 64)), dim3(64), 0, st, NG, N, pm, cl, cr);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sigma, dim3(NG), dim3(256), 0, st, looks, NG, N, sig);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_slope_weights, dim3(1), dim3(256), 0, st, NA, p.sigma_span, om);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_table, dim3(ceil_div((int64_t)NG * NAl, 128)), dim3(128), 0, st, NG, NAl,
                       N, NA, p.sigma_span, pm, cl, cr, sig, om, lut_dev);
    WW_LAUNCH_CHECK();
    WW_HIP(hipStreamSynchronize(st));
    return WW_OK;
}

// The table at a non-integer number of looks l0 + f / 2^16: the tables of
// the two neighbouring integers blended entry by entry in 2^-16 fixed point,
// rounded down (the interpolation over L of Section II-B's table grid).
__global__ void k_lut_blend_looks(const int16_t *__restrict__ T0, const int16_t *__restrict__ T1,
                                  int64_t n, int f, int16_t *__restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (int16_t)(((int64_t)T0[k] * (65536 - f) + (int64_t)T1[k] * f) >> 16);
}

ww_status blend_lut_looks(const int16_t *T0, const int16_t *T1, int64_t n, int f, int16_t *out,
                          hipStream_t stream) {
    hipLaunchKernelGGL(k_lut_blend_looks, dim3(ceil_div(n, 256)), dim3(256), 0, stream, T0, T1, n, f, out);
    WW_LAUNCH_CHECK();
    return WW_OK;
}

}  // namespace ww
