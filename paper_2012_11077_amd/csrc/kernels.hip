// HIP kernels of libcfar2d.so for gfx950 (CDNA4, wave64).
//
// Method: Rohman, Andra, Nishimoto, arXiv 2012.11077, Sec. II.B.
//   eq. (3) integral image, eq. (4) four-corner rectangle sums, eq. (2)
//   threshold T = alpha * A with alpha = N (Pfa^(-1/N) - 1), eq. (1) CUT > T.
//
// Kernels
//   sat_aggregate / sat_carry_rows / sat_carry_cols / sat_finalize
//       PLAIN integral image in three steps: per-tile aggregates, carries
//       scanned across tiles, then each tile re-reads X and writes S.
//   stencil_plain
//       eight corners of eq. (4) read from the FP64 integral image.
//   lut_kernel
//       per-map table beta(n) = alpha(n)/n = expm1(-ln(Pfa)/n) for clipped
//       border windows (NaN at n = 0: no training cells, no detection); also
//       zeroes the work counters of the fused kernels.
//   stencil_direct
//       DIRECT form (the comparison route of Table I): every cell sums its
//       own training cells from an LDS tile, no integral image.
// (The TILED form's fused kernel is in fused.hip, detection lists and packed
// masks in detections.hip, the map built from a raw record in mapbuild.hip.)
#include "internal.h"

#include <cmath>
#include <type_traits>

namespace cfar {

// ---------------------------------------------------------------------------
// Wave64 primitives on doubles (DPP on the two 32-bit halves).
// ---------------------------------------------------------------------------
namespace dpp {
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kWaveShr1 = 0x138, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
}  // namespace dpp

template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffll);
    int hi = (int)(b >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, BANK_MASK, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, BANK_MASK, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Inclusive prefix sum within each 32-lane half of the wave.
__device__ __forceinline__ double seg32_incl_scan(double v)
{
    v += dpp_f64<dpp::kRowShr1>(v);
    v += dpp_f64<dpp::kRowShr2>(v);
    v += dpp_f64<dpp::kRowShr4>(v);
    v += dpp_f64<dpp::kRowShr8>(v);
    v += dpp_f64<dpp::kRowBcast15, 0xa>(v);
    return v;
}

// Inclusive prefix sum over the 64 lanes of the wave (all lanes active).
__device__ __forceinline__ double wave_incl_scan(double v)
{
    v = seg32_incl_scan(v);
    v += dpp_f64<dpp::kRowBcast31, 0xc>(v);
    return v;
}

// dpp_f64 into `old`: lanes of rows that ROW_MASK leaves out keep old's value.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64_into(double old, double v)
{
    const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
    int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// wave_incl_scan for a loop: z15 and z31 are carried from call to call (0.0
// before the first); the rows their broadcast steps leave out stay zero in
// them, so those steps need no zeroed register each time.
__device__ __forceinline__ double wave_incl_scan_carried(double v, double &z15, double &z31)
{
    v += dpp_f64<dpp::kRowShr1>(v);
    v += dpp_f64<dpp::kRowShr2>(v);
    v += dpp_f64<dpp::kRowShr4>(v);
    v += dpp_f64<dpp::kRowShr8>(v);
    z15 = dpp_f64_into<dpp::kRowBcast15, 0xa>(z15, v);
    v += z15;
    z31 = dpp_f64_into<dpp::kRowBcast31, 0xc>(z31, v);
    v += z31;
    return v;
}

// Value of the previous lane (0 for lane 0).
__device__ __forceinline__ double wave_shift_up1(double v) { return dpp_f64<dpp::kWaveShr1>(v); }

__device__ __forceinline__ double wave_bcast_last(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T>
__device__ __forceinline__ double ld_x(const T *p) { return (double)(*p); }

// ---------------------------------------------------------------------------
// PLAIN integral image (eq. 3).  Tiles of 32 rows x 256 columns; one thread
// per tile column.  S(i,j) = top(j) + sum_{r0<=i'<=i} [left(i') + p(i',j)]
// with p the row prefix inside the tile, left(i) the sum of X(i, .) left of
// the tile and top(j) = S(r0-1, j).
// ---------------------------------------------------------------------------

// Block-wide (256 threads) inclusive prefix of one double per thread.
// `wtot` holds 2 x 4 doubles of LDS; `parity` alternates between calls so a
// single barrier per call suffices.
__device__ __forceinline__ double block_incl_scan256(double v, double *wtot, int parity, double *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s = wave_incl_scan(v);
    double *slot = wtot + parity * 4;
    if (lane == 63) slot[wave] = s;
    __syncthreads();
    double off = 0.0;
    for (int w = 0; w < wave; ++w) off += slot[w];
    if (total) *total = slot[0] + slot[1] + slot[2] + slot[3];
    return off + s;
}

template <typename T>
__global__ void __launch_bounds__(256) sat_aggregate(const T *__restrict__ x, int64_t R, int64_t F, int64_t ld,
                                                     SatWs ws)
{
    __shared__ double rowpart[kSatTH][4];
    __shared__ double wtot[8];
    const int64_t J = blockIdx.x % ws.nJ, I = blockIdx.x / ws.nJ;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t j = J * kSatTW + t;
    const int64_t r0 = I * kSatTH;
    double colsum = 0.0;
    for (int il = 0; il < kSatTH; ++il) {
        const int64_t i = r0 + il;
        double v = 0.0;
        if (i < R && j < F) v = ld_x(x + i * ld + j);
        colsum += v;
        // wave total of this row -> lane 63
        const double s = wave_incl_scan(v);
        if (lane == 63) rowpart[il][wave] = s;
    }
    double tot;
    const double cs = block_incl_scan256(colsum, wtot, 0, &tot);  // syncs: rowpart is complete too
    const int64_t tile = I * ws.nJ + J;
    ws.agg_cs[tile * kSatTW + t] = cs;
    if (t < kSatTH)
        ws.agg_row[tile * kSatTH + t] = ((rowpart[t][0] + rowpart[t][1]) + rowpart[t][2]) + rowpart[t][3];
    if (t == 0) ws.agg_tot[tile] = tot;
}

// left[I][J][il] = sum_{J'<J} agg_row[I][J'][il];  rt[I][J] = sum_{J'<J} agg_tot[I][J']
__global__ void __launch_bounds__(256) sat_carry_rows(SatWs ws)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over nI * 32 rows
    if (g >= ws.nI * kSatTH) return;
    const int64_t I = g / kSatTH;
    const int il = (int)(g % kSatTH);
    double run = 0.0, runt = 0.0;
    for (int64_t J = 0; J < ws.nJ; ++J) {
        const int64_t tile = I * ws.nJ + J;
        ws.left[tile * kSatTH + il] = run;
        run += ws.agg_row[tile * kSatTH + il];
        if (il == 0) {
            ws.rt[tile] = runt;
            runt += ws.agg_tot[tile];
        }
    }
}

// top[I][J][jl] = sum_{I'<I} (agg_cs[I'][J][jl] + rt[I'][J])  = S(32 I - 1, 256 J + jl)
__global__ void __launch_bounds__(256) sat_carry_cols(SatWs ws)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over nJ * 256 columns
    if (g >= ws.nJ * kSatTW) return;
    const int64_t J = g / kSatTW;
    const int jl = (int)(g % kSatTW);
    double run = 0.0;
    for (int64_t I = 0; I < ws.nI; ++I) {
        const int64_t tile = I * ws.nJ + J;
        ws.top[tile * kSatTW + jl] = run;
        run += ws.agg_cs[tile * kSatTW + jl] + ws.rt[tile];
    }
}

// OUT_FORM 0: FP64 S, ld = F.  OUT_FORM 1: TILED layout (FP32 local 32x32
// sums + FP64 row lines every 32 rows + FP64 column lines every 32 columns).
template <typename T, int OUT_FORM>
__global__ void __launch_bounds__(256) sat_finalize(const T *__restrict__ x, int64_t R, int64_t F, int64_t ld,
                                                    SatWs ws, double *__restrict__ s_out,
                                                    float *__restrict__ loc_out, double *__restrict__ rowline,
                                                    double *__restrict__ colline)
{
    __shared__ double wtot[8];
    const int64_t J = blockIdx.x % ws.nJ, I = blockIdx.x / ws.nJ;
    const int t = threadIdx.x;
    const int64_t j = J * kSatTW + t;
    const int64_t r0 = I * kSatTH;
    const int64_t tile = I * ws.nJ + J;
    double s_run = ws.top[tile * kSatTW + t];
    double loc_run = 0.0;
    if (OUT_FORM == 1 && j < F) rowline[(r0 / kLine) * F + j] = s_run;
    const int64_t nJ32 = (F + kLine - 1) / kLine;
    for (int il = 0; il < kSatTH; ++il) {
        const int64_t i = r0 + il;
        if (i >= R) break;  // uniform across the block
        double v = 0.0;
        if (j < F) v = ld_x(x + i * ld + j);
        double seg = 0.0;
        if (OUT_FORM == 1) seg = seg32_incl_scan(v);
        const double p = block_incl_scan256(v, wtot, il & 1, nullptr);
        s_run += ws.left[tile * kSatTH + il] + p;
        if (OUT_FORM == 0) {
            if (j < F) s_out[i * F + j] = s_run;
        } else {
            loc_run += seg;
            if (j < F) loc_out[i * F + j] = (float)loc_run;
            // column line J32 = (j+1)/32 holds S(i, 32*J32 - 1)
            if (((j + 1) % kLine) == 0 && (j + 1) / kLine < nJ32) colline[((j + 1) / kLine) * R + i] = s_run;
            if (j == 0) colline[i] = 0.0;
        }
    }
}

hipError_t launch_sat2d(const void *x, int dtype, int64_t rows, int64_t cols, int64_t ld, int out_form,
                        void *sat, const SatWs &ws, hipStream_t stream)
{
    const dim3 grid((unsigned)(ws.nJ * ws.nI));
    if (dtype == 0)
        hipLaunchKernelGGL(sat_aggregate<float>, grid, dim3(256), 0, stream, (const float *)x, rows, cols, ld, ws);
    else
        hipLaunchKernelGGL(sat_aggregate<double>, grid, dim3(256), 0, stream, (const double *)x, rows, cols, ld, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const int64_t n = ws.nI * kSatTH;
        hipLaunchKernelGGL(sat_carry_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ws);
    }
    {
        const int64_t n = ws.nJ * kSatTW;
        hipLaunchKernelGGL(sat_carry_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ws);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double *s_out = nullptr, *rowline = nullptr, *colline = nullptr;
    float *loc = nullptr;
    if (out_form == 0) {
        s_out = (double *)sat;
    } else {
        char *base = (char *)sat;
        const size_t loc_bytes = align_up((size_t)rows * (size_t)cols * 4, 256);
        const int64_t nI32 = (rows + kLine - 1) / kLine;
        const size_t row_bytes = align_up((size_t)nI32 * (size_t)cols * 8, 256);
        loc = (float *)base;
        rowline = (double *)(base + loc_bytes);
        colline = (double *)(base + loc_bytes + row_bytes);
    }
#define CFAR_SAT_FIN(T, F_)                                                                                   \
    hipLaunchKernelGGL((sat_finalize<T, F_>), grid, dim3(256), 0, stream, (const T *)x, rows, cols, ld, ws, \
                       s_out, loc, rowline, colline)
    if (dtype == 0) {
        if (out_form == 0) CFAR_SAT_FIN(float, 0); else CFAR_SAT_FIN(float, 1);
    } else {
        if (out_form == 0) CFAR_SAT_FIN(double, 0); else CFAR_SAT_FIN(double, 1);
    }
#undef CFAR_SAT_FIN
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Threshold tables (eq. 2): lut[n] = expm1(-ln(Pfa)/n) = alpha(n) / n.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) lut_kernel(const char *__restrict__ descs, uint32_t stride, MapDesc single,
                                                  uint32_t *counter)
{
    if (blockIdx.x == 0 && threadIdx.x < 16 && counter) counter[threadIdx.x] = 0u;
    const MapDesc *d = descs ? (const MapDesc *)(descs + (size_t)blockIdx.x * stride) : &single;
    double *lut = d->lut;
    const double nl = d->neg_log_pfa;
    const int n_full = d->n_full;
    for (int n = threadIdx.x; n <= n_full; n += blockDim.x)
        lut[n] = n == 0 ? __builtin_nan("") : expm1(nl / (double)n);
}

hipError_t launch_lut(const void *descs, size_t stride, const MapDesc &single, int n, uint32_t *counter,
                      hipStream_t stream)
{
    hipLaunchKernelGGL(lut_kernel, dim3((unsigned)(descs ? n : 1)), dim3(256), 0, stream, (const char *)descs,
                       (uint32_t)stride, single, counter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Clipped window sizes and the decision, shared by both stencils.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clip_len(int c, int h, int n)
{
    const int lo = c - h < 0 ? 0 : c - h;
    const int hi = c + h > n - 1 ? n - 1 : c + h;
    return hi - lo + 1;
}

// ---------------------------------------------------------------------------
// PLAIN stencil: eq. (4) twice on the FP64 integral image, one thread per cell.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) stencil_plain(MapDesc d, const double *__restrict__ S)
{
    const int ncb = (d.cols + 255) / 256;
    const int i = (int)(blockIdx.x / (unsigned)ncb);
    const int j = (int)(blockIdx.x % (unsigned)ncb) * 256 + threadIdx.x;
    if (j >= d.cols) return;
    const int R = d.rows, F = d.cols;
    auto at = [&](int r, int c) -> double { return (r < 0 || c < 0) ? 0.0 : S[(int64_t)r * F + c]; };
    const int ro0 = max(0, i - d.hr), ro1 = min(R - 1, i + d.hr);
    const int co0 = max(0, j - d.hf), co1 = min(F - 1, j + d.hf);
    const int ri0 = max(0, i - d.gr), ri1 = min(R - 1, i + d.gr);
    const int ci0 = max(0, j - d.gf), ci1 = min(F - 1, j + d.gf);
    // eq. (4): A = L1 + L4 - (L2 + L3); L1 outside top-left, L4 inclusive bottom-right
    const double outer = at(ro0 - 1, co0 - 1) + at(ro1, co1) - (at(ro0 - 1, co1) + at(ro1, co0 - 1));
    const double inner = at(ri0 - 1, ci0 - 1) + at(ri1, ci1) - (at(ri0 - 1, ci1) + at(ri1, ci0 - 1));
    const double st = outer - inner;
    const int nt = (ro1 - ro0 + 1) * (co1 - co0 + 1) - (ri1 - ri0 + 1) * (ci1 - ci0 + 1);
    const double cut = ld_x((const T *)d.x + (int64_t)i * d.ld + j);
    const double thr = nt > 0 ? d.lut[nt] * st : INFINITY;
    const int64_t o = (int64_t)i * d.ld_mask + j;
    d.mask[o] = (uint8_t)(nt > 0 && cut > thr);
    if (d.train_sum) d.train_sum[o] = st;
    if (d.thresh) d.thresh[o] = thr;
}

hipError_t launch_stencil_plain(const MapDesc &d, const double *sat, hipStream_t stream)
{
    const dim3 grid((unsigned)(((int64_t)d.cols + 255) / 256 * d.rows));
    if (d.dtype == 0)
        hipLaunchKernelGGL(stencil_plain<float>, grid, dim3(256), 0, stream, d, sat);
    else
        hipLaunchKernelGGL(stencil_plain<double>, grid, dim3(256), 0, stream, d, sat);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// DIRECT form: CA-CFAR without the integral image (the comparison route of
// Table I): every cell sums its own training cells.  A workgroup of four
// waves owns kDirTH x kDirTW outputs (wave w: row i0 + w, lane: column
// j0 + lane); the tile and its halo of hr rows and hf columns are staged in
// LDS in the map's type, cells outside the map as zero (the clipped sum).
// Along a window row the guard test is the same for the whole wave.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) stencil_direct(MapDesc d)
{
    extern __shared__ char direct_lds[];
    T *tile = (T *)direct_lds;
    const int R = d.rows, F = d.cols, hr = d.hr, hf = d.hf, gr = d.gr, gf = d.gf;
    const int tcols = kDirTW + 2 * hf, trows = kDirTH + 2 * hr;
    const int nbj = (F + kDirTW - 1) / kDirTW;
    const int i0 = (int)(blockIdx.x / (unsigned)nbj) * kDirTH;
    const int j0 = (int)(blockIdx.x % (unsigned)nbj) * kDirTW;
    const T *__restrict__ X = (const T *)d.x;
    for (int t = threadIdx.x; t < trows * tcols; t += 256) {
        const int a = t / tcols, b = t - a * tcols;
        const int r = i0 - hr + a, c = j0 - hf + b;
        tile[t] = (r >= 0 && r < R && c >= 0 && c < F) ? X[(int64_t)r * d.ld + c] : (T)0;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = i0 + w, j = j0 + lane;
    // four partial sums break the chain of dependent FP64 adds
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto run = [&](const T *p, int n) {  // p[0 .. n-1]
        int c = 0;
        for (; c + 4 <= n; c += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += (double)p[c + u];
        }
        for (; c < n; ++c) acc[0] += (double)p[c];
    };
    for (int da = -hr; da <= hr; ++da) {
        const T *row = tile + (w + hr + da) * tcols + lane;  // column j - hf
        if (da >= -gr && da <= gr) {                           // guard band: both sides of the guard
            run(row, hf - gf);
            run(row + hf + gf + 1, hf - gf);
        } else {
            run(row, 2 * hf + 1);
        }
    }
    if (i >= R || j >= F) return;
    const double st = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    const int nt = clip_len(i, hr, R) * clip_len(j, hf, F) - clip_len(i, gr, R) * clip_len(j, gf, F);
    const double cut = ld_x(X + (int64_t)i * d.ld + j);
    const double thr = nt > 0 ? d.lut[nt] * st : INFINITY;
    const int64_t o = (int64_t)i * d.ld_mask + j;
    d.mask[o] = (uint8_t)(nt > 0 && cut > thr);
    if (d.train_sum) d.train_sum[o] = st;
    if (d.thresh) d.thresh[o] = thr;
}

size_t direct_lds_bytes(int hr, int hf, int dtype)
{
    return (size_t)(kDirTH + 2 * hr) * (size_t)(kDirTW + 2 * hf) * (dtype == 0 ? 4 : 8);
}

hipError_t launch_stencil_direct(const MapDesc &d, hipStream_t stream)
{
    const int64_t nb = ((int64_t)d.rows + kDirTH - 1) / kDirTH * (((int64_t)d.cols + kDirTW - 1) / kDirTW);
    const size_t lds = direct_lds_bytes(d.hr, d.hf, d.dtype);
    if (d.dtype == 0)
        hipLaunchKernelGGL(stencil_direct<float>, dim3((unsigned)nb), dim3(256), lds, stream, d);
    else
        hipLaunchKernelGGL(stencil_direct<double>, dim3((unsigned)nb), dim3(256), lds, stream, d);
    return hipGetLastError();
}

}  // namespace cfar
