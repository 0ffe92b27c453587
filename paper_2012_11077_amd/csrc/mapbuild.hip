// The primary signal processing of Sec. II.A on the GPU: from a raw record
// (N traces of M fast-time samples, stored trace by trace) to the range x
// slow-time-frequency power map that CA-CFAR runs on.
//   mb_coef:      per trace, the mean and the least-squares slope over the
//                 sample index (DC-shift removal + linear-trend subtraction);
//   mb_transpose: the detrended record, range-major (rows = range bins,
//                 slow time contiguous), FP64, through an LDS tile;
//   mb_twiddle:   the N roots of unity, once;
//   mb_band:      per range bin (one workgroup): the centred mean filter of
//                 odd length L along slow time, the record's largest
//                 magnitude (atomic maximum), and the DFT of the band's bins
//                 (root index (k n) mod N, kept exactly in integers), power
//                 re^2 + im^2;
//   mb_scale:     normalisation by the largest magnitude (power / max^2) into
//                 the output map's type.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace cfar {

constexpr int kMbMaxTraces = 4000;  // one range bin's slow-time row (two FP64 copies) in 64 KB of LDS

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
__global__ void __launch_bounds__(256) mb_coef(const T *__restrict__ raw, int64_t M, int64_t ld,
                                               double *__restrict__ coef, unsigned long long *__restrict__ gmax)
{
    __shared__ double s0w[4], s1w[4];
    const int64_t n = blockIdx.x;
    const T *y = raw + n * ld;
    const double tm = 0.5 * (double)(M - 1);
    double s0 = 0.0, s1 = 0.0;
    for (int64_t t = threadIdx.x; t < M; t += 256) {
        const double v = (double)y[t];
        s0 += v;
        s1 += ((double)t - tm) * v;
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s0w[w] = s0;
        s1w[w] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double S0 = (s0w[0] + s0w[1]) + (s0w[2] + s0w[3]);
        const double S1 = (s1w[0] + s1w[1]) + (s1w[2] + s1w[3]);
        const double Md = (double)M;
        const double stt = Md * (Md * Md - 1.0) / 12.0;  // sum of (t - tm)^2
        coef[2 * n] = S0 / Md;
        coef[2 * n + 1] = stt > 0.0 ? S1 / stt : 0.0;
        if (n == 0) *gmax = 0ull;
    }
}

// Tile: 64 samples (m) x 16 traces (n).
template <typename T>
__global__ void __launch_bounds__(256) mb_transpose(const T *__restrict__ raw, int64_t N, int64_t M, int64_t ld,
                                                    const double *__restrict__ coef, double *__restrict__ D)
{
    __shared__ double tile[16][65];
    const int64_t nbm = (M + 63) / 64;
    const int64_t m0 = (int64_t)(blockIdx.x % (unsigned)nbm) * 64;
    const int64_t n0 = (int64_t)(blockIdx.x / (unsigned)nbm) * 16;
    const double tm = 0.5 * (double)(M - 1);
    const int j = threadIdx.x & 63;
    for (int i = threadIdx.x >> 6; i < 16; i += 4) {
        const int64_t n = n0 + i, m = m0 + j;
        double v = 0.0;
        if (n < N && m < M) v = (double)raw[n * ld + m] - (coef[2 * n] + coef[2 * n + 1] * ((double)m - tm));
        tile[i][j] = v;
    }
    __syncthreads();
    const int i = threadIdx.x & 15;
    for (int jj = threadIdx.x >> 4; jj < 64; jj += 16) {
        const int64_t n = n0 + i, m = m0 + jj;
        if (n < N && m < M) D[m * N + n] = tile[i][jj];
    }
}

// The N roots of unity once: tw[2r], tw[2r+1] = cos, sin of 2 pi r / N.
__global__ void __launch_bounds__(256) mb_twiddle(int N, double *__restrict__ tw)
{
    for (int r = blockIdx.x * 256 + threadIdx.x; r < N; r += gridDim.x * 256) {
        double sn, cs;
        sincospi(2.0 * (double)r / (double)N, &sn, &cs);
        tw[2 * r] = cs;
        tw[2 * r + 1] = sn;
    }
}

__global__ void __launch_bounds__(256) mb_band(const double *__restrict__ D, int N, int L, int k0, int nb,
                                               const double *__restrict__ tw, double *__restrict__ P,
                                               unsigned long long *__restrict__ gmax)
{
    extern __shared__ double mb_lds[];
    double *d = mb_lds;       // N
    double *g = mb_lds + N;   // N
    __shared__ double wmax[4];
    const int64_t m = blockIdx.x;
    for (int n = threadIdx.x; n < N; n += 256) d[n] = D[m * N + n];
    __syncthreads();
    const int h = L / 2;
    double amax = 0.0;
    for (int n = threadIdx.x; n < N; n += 256) {
        const int lo = n - h < 0 ? 0 : n - h, hi = n + h > N - 1 ? N - 1 : n + h;
        double s = 0.0;
        for (int q = lo; q <= hi; ++q) s += d[q];
        const double v = s / (double)(hi - lo + 1);
        g[n] = v;
        amax = fmax(amax, fabs(v));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) wmax[w] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        // non-negative doubles order like their bit patterns
        atomicMax(gmax, (unsigned long long)__double_as_longlong(mx));
    }
    for (int b = w; b < nb; b += 4) {
        const int64_t k = k0 + b;
        double re = 0.0, im = 0.0;
        // root index r = (k n) mod N, advanced by (64 k) mod N per step; the
        // root itself is rotated by the step's root and taken afresh from
        // the table every 16 steps (rounding stays near 1e-15)
        const int step = (int)((64 * k) % N);
        const double sc = tw[2 * step], ss = tw[2 * step + 1];
        int r = (int)((k * (int64_t)lane) % N);
        double wc = 0.0, ws = 0.0;
        int i = 0;
        for (int n = lane; n < N; n += 64, ++i) {
            if ((i & 15) == 0) {
                wc = tw[2 * r];
                ws = tw[2 * r + 1];
            }
            re += g[n] * wc;
            im -= g[n] * ws;
            const double c2 = wc * sc - ws * ss;
            ws = ws * sc + wc * ss;
            wc = c2;
            r += step;
            if (r >= N) r -= N;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) P[m * nb + b] = re * re + im * im;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) mb_scale(const double *__restrict__ P, int64_t M, int nb,
                                                const unsigned long long *__restrict__ gmax, T *__restrict__ out,
                                                int64_t ld_out)
{
    const double mx = __longlong_as_double((long long)*gmax);
    const double s = mx > 0.0 ? 1.0 / (mx * mx) : 0.0;
    const int64_t total = M * nb;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t m = i / nb, b = i - m * nb;
        out[m * ld_out + b] = (T)(P[i] * s);
    }
}

static int mb_bins(int64_t n_traces, const cfar_mapbuild_params *p, int32_t *k0, int32_t *nb)
{
    if (!p) return set_error(CFAR_EINVAL, "params is NULL");
    if (n_traces < 1 || n_traces > kMbMaxTraces)
        return set_error(CFAR_EINVAL, "n_traces must lie in [1, %d]", kMbMaxTraces);
    if (!(p->fs_slow > 0.0) || !std::isfinite(p->fs_slow)) return set_error(CFAR_EINVAL, "fs_slow must be > 0");
    if (!(p->f_lo >= 0.0) || !(p->f_hi >= p->f_lo) || !std::isfinite(p->f_hi))
        return set_error(CFAR_EINVAL, "need 0 <= f_lo <= f_hi");
    const double N = (double)n_traces;
    const int64_t a = (int64_t)std::ceil(p->f_lo * N / p->fs_slow - 1e-9);
    const int64_t b = std::min<int64_t>((int64_t)std::floor(p->f_hi * N / p->fs_slow + 1e-9), n_traces / 2);
    if (b < a) return set_error(CFAR_EINVAL, "the band [f_lo, f_hi] holds no DFT bin of %lld traces", (long long)n_traces);
    *k0 = (int32_t)a;
    *nb = (int32_t)(b - a + 1);
    return CFAR_OK;
}

struct MbLayout {
    size_t coef, tw, D, P, gmax, total;
};

static MbLayout mb_layout(int64_t N, int64_t M, int64_t nb)
{
    MbLayout L;
    L.coef = 0;
    L.tw = align_up((size_t)N * 16, 256);
    L.D = L.tw + align_up((size_t)N * 16, 256);
    L.P = L.D + align_up((size_t)M * (size_t)N * 8, 256);
    L.gmax = L.P + align_up((size_t)M * (size_t)nb * 8, 256);
    L.total = L.gmax + 256;
    return L;
}

}  // namespace cfar

using namespace cfar;

extern "C" {

int cfar_map_bins(int64_t n_traces, const cfar_mapbuild_params *params, int32_t *first_bin, int32_t *n_bins)
{
    if (!first_bin || !n_bins) return set_error(CFAR_EINVAL, "first_bin or n_bins is NULL");
    return mb_bins(n_traces, params, first_bin, n_bins);
}

size_t cfar_map_build_workspace_bytes(int64_t n_traces, int64_t n_samples, const cfar_mapbuild_params *params)
{
    int32_t k0, nb;
    if (mb_bins(n_traces, params, &k0, &nb) != CFAR_OK) return 0;
    if (n_samples < 1 || n_samples > (int64_t(1) << 30)) return 0;
    return mb_layout(n_traces, n_samples, nb).total;
}

int cfar_map_build(const void *raw, int32_t raw_dtype, int64_t n_traces, int64_t n_samples, int64_t ld_raw,
                   const cfar_mapbuild_params *params, void *map_out, int64_t ld_map, void *ws, size_t ws_bytes,
                   void *stream)
{
    int32_t k0, nb;
    int rc = mb_bins(n_traces, params, &k0, &nb);
    if (rc != CFAR_OK) return rc;
    if (raw_dtype != CFAR_F32 && raw_dtype != CFAR_F64) return set_error(CFAR_EINVAL, "unknown raw dtype %d", raw_dtype);
    if (params->out_dtype != CFAR_F32 && params->out_dtype != CFAR_F64)
        return set_error(CFAR_EINVAL, "unknown out_dtype %d", params->out_dtype);
    if (params->mean_len < 1 || params->mean_len % 2 == 0 || params->mean_len > 1023)
        return set_error(CFAR_EINVAL, "mean_len must be odd and in [1, 1023]");
    if (n_samples < 1 || n_samples > (int64_t(1) << 30)) return set_error(CFAR_EINVAL, "n_samples must lie in [1, 2^30]");
    if (ld_raw < n_samples) return set_error(CFAR_EINVAL, "ld_raw < n_samples");
    if (ld_map < nb) return set_error(CFAR_EINVAL, "ld_map < number of band bins (%d)", nb);
    if (!raw || !map_out || !ws) return set_error(CFAR_EINVAL, "NULL pointer argument");
    const int64_t N = n_traces, M = n_samples;
    const int64_t tiles = ((M + 63) / 64) * ((N + 15) / 16);
    if (M > INT32_MAX || tiles > INT32_MAX) return set_error(CFAR_EINVAL, "record too large");
    const MbLayout L = mb_layout(N, M, nb);
    if (ws_bytes < L.total) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, L.total);
    char *base = (char *)ws;
    double *coef = (double *)(base + L.coef);
    double *tw = (double *)(base + L.tw);
    double *D = (double *)(base + L.D);
    double *P = (double *)(base + L.P);
    unsigned long long *gmax = (unsigned long long *)(base + L.gmax);
    hipStream_t s = (hipStream_t)stream;
    if (raw_dtype == CFAR_F32) {
        hipLaunchKernelGGL(mb_coef<float>, dim3((unsigned)N), dim3(256), 0, s, (const float *)raw, M, ld_raw, coef, gmax);
        hipLaunchKernelGGL(mb_transpose<float>, dim3((unsigned)tiles), dim3(256), 0, s, (const float *)raw, N, M,
                           ld_raw, (const double *)coef, D);
    } else {
        hipLaunchKernelGGL(mb_coef<double>, dim3((unsigned)N), dim3(256), 0, s, (const double *)raw, M, ld_raw, coef,
                           gmax);
        hipLaunchKernelGGL(mb_transpose<double>, dim3((unsigned)tiles), dim3(256), 0, s, (const double *)raw, N, M,
                           ld_raw, (const double *)coef, D);
    }
    hipLaunchKernelGGL(mb_twiddle, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, (int)N, tw);
    hipLaunchKernelGGL(mb_band, dim3((unsigned)M), dim3(256), (size_t)(2 * N * 8), s, (const double *)D, (int)N,
                       (int)params->mean_len, (int)k0, (int)nb, (const double *)tw, P, gmax);
    const unsigned g = (unsigned)std::min<int64_t>((M * nb + 255) / 256, 65536);
    if (params->out_dtype == CFAR_F32)
        hipLaunchKernelGGL(mb_scale<float>, dim3(g), dim3(256), 0, s, (const double *)P, M, (int)nb,
                           (const unsigned long long *)gmax, (float *)map_out, ld_map);
    else
        hipLaunchKernelGGL(mb_scale<double>, dim3(g), dim3(256), 0, s, (const double *)P, M, (int)nb,
                           (const unsigned long long *)gmax, (double *)map_out, ld_map);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "launch(map build)");
    return CFAR_OK;
}

}  // extern "C"
