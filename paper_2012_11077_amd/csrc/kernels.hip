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
//       border windows; also zeroes the work counters of the fused kernels.
//   fused_kernel
//       TILED form: persistent, one wave per work unit (a strip of 64*K
//       columns x rs rows of one map).  The eight corners of eq. (4) are taken
//       in two separable steps: FP64 running column sums over the outer and
//       inner window rows hold the four row corners, a wave-wide FP64 row
//       prefix of those column sums gives the four column corners as
//       differences read back from LDS.  The integral image itself is never
//       written; one pass over X.
//   stencil_direct
//       DIRECT form (the comparison route of Table I): every cell sums its
//       own training cells from an LDS tile, no integral image.
// (Detection lists and packed masks are in detections.hip, the map built
// from a raw record in mapbuild.hip.)
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
__global__ void __launch_bounds__(256) lut_kernel(const MapDesc *__restrict__ descs, MapDesc single,
                                                  uint32_t *counter)
{
    if (blockIdx.x == 0 && threadIdx.x < 16 && counter) counter[threadIdx.x] = 0u;
    const MapDesc *d = descs ? descs + blockIdx.x : &single;
    double *lut = d->lut;
    const double nl = d->neg_log_pfa;
    const int n_full = d->n_full;
    for (int n = threadIdx.x; n <= n_full; n += blockDim.x)
        lut[n] = n == 0 ? 0.0 : expm1(nl / (double)n);
}

hipError_t launch_lut(const MapDesc *descs, const MapDesc &single, int n, uint32_t *counter, hipStream_t stream)
{
    hipLaunchKernelGGL(lut_kernel, dim3((unsigned)(descs ? n : 1)), dim3(256), 0, stream, descs, single, counter);
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

// ---------------------------------------------------------------------------
// TILED form: persistent fused kernel, one instantiation per (K, T).
//
// One wave owns a work unit: a strip of W = 64*K map columns (the strip's
// output columns plus a halo of H >= hf + 1 columns on each side; lane l
// holds columns l*K .. l*K+K-1 of the strip) and rs output rows.  Per output
// row r:
//   1. two FP64 running column sums of the strip, over rows r-hr .. r+hr
//      (outer window) and r-gr .. r+gr (inner window), each step adding the
//      row that enters and taking off the row that leaves: the row corners
//      of eq. (4);
//   2. an FP64 row prefix of those column sums across the strip (in-lane
//      serial over K columns, then a DPP scan over the 64 lanes);
//   3. the column corners of eq. (4): prefix differences at p + h and
//      p - h - 1, read back from LDS;
//   4. training sum, N, T = beta(N) * sum, decision, mask store.
// The next row's loads are issued before the current row is processed.
// ---------------------------------------------------------------------------

// Global-memory pointers (address space 1): descriptors hand the kernels
// generic pointers, which would otherwise compile to flat accesses.
#define CFAR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const CFAR_GLOBAL T *gbl(const T *p) { return (const CFAR_GLOBAL T *)p; }
template <typename T>
__device__ __forceinline__ CFAR_GLOBAL T *gbl_w(T *p) { return (CFAR_GLOBAL T *)p; }

// Work-unit modes of the TILED kernel.  FAST: every lane's K columns lie
// inside the map.  EDGE: a lane's K columns lie all inside or all outside the
// map (a strip at the left or right border).  GENERAL: anything else.
enum { kGeneral = 0, kEdge = 1, kFast = 2 };

// Loads of K consecutive values of one row (row: wave-uniform byte pointer)
// starting at strip column c.  FAST: vector load.  EDGE: vector load, from
// column 0 (F >= K) for a lane outside the map (`out`), whose values the
// caller then weighs by zero where they are used (a select here would make
// the load wait at once).  GENERAL: each column clamped into [0, F) and
// zeroed outside, so every access stays in bounds.
template <int K, typename T, int MODE>
__device__ __forceinline__ void ldk(const CFAR_GLOBAL char *row, int c, int F, bool out, T (&v)[K])
{
    if constexpr ((MODE & 3) != kGeneral) {
        const uint32_t off = (MODE & 3) == kEdge && out ? 0u : (uint32_t)c * (uint32_t)sizeof(T);
        // K values in one (or two) vector loads, stated as unaligned copies:
        // rows need not be 16-byte aligned (the memory runs in
        // unaligned-access mode)
        if constexpr (K * sizeof(T) == 8) {
            __builtin_memcpy((char *)v, (const char *)(row + off), 8);
        } else {
#pragma unroll
            for (int q = 0; q < (int)(K * sizeof(T) / 16); ++q)
                __builtin_memcpy((char *)v + 16 * q, (const char *)(row + off + 16u * q), 16);
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int cc = c + k;
            const int cl = min(max(cc, 0), F - 1);
            const T t = *(const CFAR_GLOBAL T *)(row + (uint32_t)cl * (uint32_t)sizeof(T));
            v[k] = (cc >= 0 && cc < F) ? t : T(0);
        }
    }
}

// acc += s * v with s = 1.0 (row entering the window), -1.0 (row leaving
// it) or 0.0 (row outside the map): branch-free, and bit-identical to
// adding, subtracting or skipping the row.
template <int K, typename T>
__device__ __forceinline__ void acc_row(double (&a)[K], const T (&v)[K], double s)
{
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = __builtin_fma(s, (double)v[k], a[k]);
}

// Lane-major LDS layout of one prefix row: position p = l*K + k at
// [k*64 + l].  Position p + o for element k of lane l, with o = q*K + s
// (0 <= s < K), is element (k+s) mod K of lane l+q, or of lane l+q+1 when
// k+s >= K.  The K addresses depend only on o and the lane, so they are
// formed once per work unit.  Lane indices wrap inside the row so every
// address stays in the wave's region (wrapped values only reach positions
// that are not outputs).
template <int K>
struct OffsetRead {
    int addr[K];
    __device__ __forceinline__ void init(int o, int lane)
    {
        const int q = o >= 0 ? o / K : -((-o + K - 1) / K);
        const int s = o - q * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = k + s;
            addr[k] = (e >= K ? e - K : e) * 64 + ((lane + q + (e >= K ? 1 : 0)) & 63);
        }
    }
    __device__ __forceinline__ double get(const double *__restrict__ q, int k) const { return q[addr[k]]; }
};

// Rows whose loads are in flight in the interior loop.
#ifndef CFAR_PREFETCH_ROWS
#define CFAR_PREFETCH_ROWS 2
#endif
template <int K, typename T>
constexpr int prefetch_rows() { return K * sizeof(T) >= 32 ? 2 : CFAR_PREFETCH_ROWS; }
#ifndef CFAR_PREFETCH_ROWS_FULL
#define CFAR_PREFETCH_ROWS_FULL 3
#endif
template <int K, typename T>
constexpr int prefetch_rows_full() { return K * sizeof(T) >= 32 ? 3 : CFAR_PREFETCH_ROWS_FULL; }
// Rows loaded together in the warm-up.
template <int K, typename T>
constexpr int warm_rows() { return K * sizeof(T) >= 32 ? 4 : 8; }
// Word 3 of a raw buffer resource on CDNA (32-bit data format, no swizzle).
constexpr int kBufferFlags = 0x00020000;

// K consecutive values of one row through a buffer resource: lane byte
// offset voff, wave-uniform row byte offset soff (any alignment of the
// element type: the memory runs in unaligned-access mode).
template <int K, typename T>
__device__ __forceinline__ void ldk_buf(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, T (&v)[K])
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    if constexpr (K * sizeof(T) == 8) {
        const u32x2 w = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
        __builtin_memcpy(v, &w, 8);
    } else {
#pragma unroll
        for (int q = 0; q < (int)(K * sizeof(T) / 16); ++q) {
            const u32x4 w = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 16u * q, soff, 0));
            __builtin_memcpy((char *)v + 16 * q, &w, 16);
        }
    }
}
// FAST units: the strip's output columns are at least hf away from both map
// borders (only rows can be clipped: N = n_full on interior rows).  EDGE
// units: a lane's K columns are all inside or all outside the map; interior
// rows clip only columns, so N and beta are fixed per lane.  In both, lanes
// hold either K output columns or none.
//
// Window sums run as two FP64 accumulators per column, the outer (rows
// r-hr .. r+hr) and the inner (rows r-gr .. r+gr) column sum: each step adds
// the row entering the window and takes off the row leaving it, the same
// value that was added, so a row outside the map (never added) is neither.
//
// Interior rows of FAST and EDGE units without the optional outputs run a
// straight-line loop (no branches, no clipping) fed through a buffer
// resource with several rows in flight; border rows, general units and maps
// with the optional outputs run a plain loop.
template <int K, typename T, int MODE, bool OUT>
__device__ void fused_unit(const MapDesc &d, int strip, int rchunk, int cs, double *__restrict__ qo,
                           double *__restrict__ qi, T *__restrict__ ring, int ring_bytes, int lane)
{
    const int R = d.rows, F = d.cols;
    const int hr = d.hr, hf = d.hf, gr = d.gr, gf = d.gf;
    const int c_out0 = strip * d.tw;
    const int c_out1 = min(c_out0 + d.tw, F);
    // cs: map column of strip position 0, c_out0 - H, or for a right-aligned
    // last strip F + H - 64K (then c_out0 - cs >= H still holds)
    const int ra = rchunk * d.rs;
    const int rb = min(ra + d.rs, R);
    const int c_lane = cs + lane * K;
    const T *__restrict__ X = (const T *)d.x;
    const int64_t ld = d.ld;

    const bool lane_any_out = (c_lane + K > c_out0) && (c_lane < c_out1);
    // first own column of the lane (0 but in a right-aligned strip, whose
    // first output column may fall inside a lane: that lane stores bytes)
    const int k_own0 = max(c_out0 - c_lane, 0);
    const bool lane_col_interior = (c_lane >= hf) && (c_lane + K - 1 + hf < F);
    // EDGE: a lane outside the map loads column 0 and weighs it by zero
    constexpr int BM = MODE & 3;  // FAST, EDGE or GENERAL
    const bool lane_outside = BM == kEdge && (c_lane < 0 || c_lane >= F);
    const double lane_w = lane_outside ? 0.0 : 1.0;
    const double beta_full = gbl(d.lut)[d.n_full];
    // EDGE: beta per lane on rows without row clipping (NaN where N = 0: no
    // detection)
    double beta_lane[BM == kEdge ? K : 1];
    if constexpr (BM == kEdge) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int jc = min(max(c_lane + k, 0), F - 1);
            const int nt = (2 * hr + 1) * clip_len(jc, hf, F) - (2 * gr + 1) * clip_len(jc, gf, F);
            beta_lane[k] = nt > 0 ? gbl(d.lut)[nt] : __builtin_nan("");
        }
    }

    OffsetRead<K> rd_oh, rd_ol, rd_ih, rd_il;
    rd_oh.init(hf, lane);
    rd_ol.init(-hf - 1, lane);
    rd_ih.init(gf, lane);
    rd_il.init(-gf - 1, lane);

    auto rowp = [&](int i) -> const CFAR_GLOBAL char * {
        const int ic = min(max(i, 0), R - 1);
        return (const CFAR_GLOBAL char *)gbl(X + (int64_t)ic * ld);
    };

    double Co[K], Ci[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { Co[k] = 0.0; Ci[k] = 0.0; }

    // Warm-up: Co over rows [ra-hr-1, ra+hr-1], Ci over rows [ra-gr-1,
    // ra+gr-1] (rows inside the map), so the first step, like every later
    // one, adds rows r+hr, r+gr and takes off rows r-hr-1, r-gr-1.
    {
        const int w0 = ra - hr - 1, w1 = ra + hr, g0 = ra - gr - 1, g1 = ra + gr;
        for (int i0 = w0; i0 < w1; i0 += warm_rows<K, T>()) {
            T w[warm_rows<K, T>()][K];
#pragma unroll
            for (int j = 0; j < warm_rows<K, T>(); ++j) ldk<K, T, MODE>(rowp(i0 + j), c_lane, F, lane_outside, w[j]);
#pragma unroll
            for (int j = 0; j < warm_rows<K, T>(); ++j) {
                const int i = i0 + j;
                const bool in = i >= 0 && i < R && i < w1;
                acc_row<K, T>(Co, w[j], in ? lane_w : 0.0);
                acc_row<K, T>(Ci, w[j], (in && i >= g0 && i < g1) ? lane_w : 0.0);
            }
        }
    }

    // Row prefix of the two column sums across the strip (in-lane serial,
    // then a DPP scan over the lanes), published in LDS: the row corners of
    // eq. (4) are in the column sums, the column corners are read back at
    // offsets +-h.
    double z15o = 0.0, z31o = 0.0, z15i = 0.0, z31i = 0.0;  // see wave_incl_scan_carried
    auto publish = [&]() {
        double po[K], pi[K];
        po[0] = Co[0];
        pi[0] = Ci[0];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            po[k] = po[k - 1] + Co[k];
            pi[k] = pi[k - 1] + Ci[k];
        }
        // exclusive prefix of the lane totals: the inclusive one minus the lane's own
        const double eo = wave_incl_scan_carried(po[K - 1], z15o, z31o) - po[K - 1];
        const double ei = wave_incl_scan_carried(pi[K - 1], z15i, z31i) - pi[K - 1];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            qo[k * 64 + lane] = eo + po[k];
            qi[k * 64 + lane] = ei + pi[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // Any row: b = rows r+hr, r+gr, r-gr-1, r-hr-1, r; rows outside the map
    // are neither added nor taken off.
    auto accumulate = [&](int r, const T(&b)[5][K]) {
        const double so = r + hr < R ? lane_w : 0.0, si = r + gr < R ? lane_w : 0.0;
        const double to = r - hr - 1 >= 0 ? -lane_w : 0.0, ti = r - gr - 1 >= 0 ? -lane_w : 0.0;
        acc_row<K, T>(Co, b[0], so);
        acc_row<K, T>(Co, b[3], to);
        acc_row<K, T>(Ci, b[1], si);
        acc_row<K, T>(Ci, b[2], ti);
        publish();
    };
    auto train_sum_at = [&](int k) -> double {
        // column corners of eq. (4): box = Q(p + h) - Q(p - h - 1), outer minus inner
        return (rd_oh.get(qo, k) - rd_ol.get(qo, k)) - (rd_ih.get(qi, k) - rd_il.get(qi, k));
    };
    // packed stores need 4-byte aligned mask rows and a strip start on a
    // multiple of min(K, 4) columns; else bytes
    const bool mvec = (d.vec_ok & 2) != 0 && (cs % (K < 4 ? K : 4)) == 0;
    auto store_bits = [&](CFAR_GLOBAL uint8_t *dst, const uint32_t(&bits)[(K + 3) / 4]) {
        if (!mvec || (BM == kEdge && k_own0 > 0)) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k >= k_own0) dst[k] = (uint8_t)(bits[k / 4] >> (8 * (k % 4)));
            return;
        }
        if constexpr (K == 2) {
            __builtin_nontemporal_store((uint16_t)bits[0], (CFAR_GLOBAL uint16_t *)dst);
        } else {
#pragma unroll
            for (int q = 0; q < K / 4; ++q) __builtin_nontemporal_store(bits[q], (CFAR_GLOBAL uint32_t *)dst + q);
        }
    };
    // Interior row of a FAST unit (N = n_full, beta = beta_full) or an EDGE
    // unit (beta per lane); every lane computes, lanes with outputs store.
    auto decide_fast = [&](const T(&xcut)[K], uint32_t(&bits)[(K + 3) / 4]) {
#pragma unroll
        for (int q = 0; q < (K + 3) / 4; ++q) bits[q] = 0u;
        // every corner read is issued before the first is used: the LDS
        // round trips overlap instead of following one another
        double oh[K], ol[K], ih[K], il[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            oh[k] = rd_oh.get(qo, k);
            ol[k] = rd_ol.get(qo, k);
            ih[k] = rd_ih.get(qi, k);
            il[k] = rd_il.get(qi, k);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double beta = BM == kEdge ? beta_lane[BM == kEdge ? k : 0] : beta_full;
            const double thr = beta * ((oh[k] - ol[k]) - (ih[k] - il[k]));
            bits[k / 4] |= ((double)xcut[k] > thr) ? (1u << (8 * (k % 4))) : 0u;
        }
    };
    auto output_fast = [&](int r, const T(&xcut)[K]) {
        uint32_t bits[(K + 3) / 4];
        decide_fast(xcut, bits);
        CFAR_GLOBAL uint8_t *mdst = gbl_w(d.mask) + (int64_t)r * d.ld_mask + c_lane;
        if (lane_any_out) store_bits(mdst, bits);
    };
    // Any row: N and beta per cell; every cell is computed, owned cells
    // store their byte.  The per-cell table loads are issued by prep() before
    // the next row's loads, so waiting for them never waits for the prefetch.
    struct Prep {
        int nt[K];
        double beta[K];
    };
    auto prep = [&](int r, Prep &pp) {
        const int nro = clip_len(r, hr, R), nri = clip_len(r, gr, R);
        const bool interior = (r >= hr) && (r + hr < R) && lane_col_interior;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int jc = min(max(c_lane + k, 0), F - 1);
            pp.nt[k] = interior ? d.n_full : nro * clip_len(jc, hf, F) - nri * clip_len(jc, gf, F);
            pp.beta[k] = gbl(d.lut)[pp.nt[k]];
        }
    };
    auto output_general = [&](int r, const T(&xcut)[K], const Prep &pp) {
        const int64_t orow = (int64_t)r * d.ld_mask;
        CFAR_GLOBAL uint8_t *mrow = gbl_w(d.mask) + orow;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double st = train_sum_at(k);
            const int j = c_lane + k;
            const double thr = pp.beta[k] * st;
            const bool own = j >= c_out0 && j < c_out1;
            if (own) mrow[j] = (uint8_t)(pp.nt[k] > 0 && (double)xcut[k] > thr);
            if constexpr (OUT) {
                if (own) {
                    if (d.train_sum) gbl_w(d.train_sum)[orow + j] = st;
                    if (d.thresh) gbl_w(d.thresh)[orow + j] = pp.nt[k] > 0 ? thr : INFINITY;
                }
            }
        }
    };
    auto issue = [&](int r, T(&b)[5][K]) {
        ldk<K, T, MODE>(rowp(r + hr), c_lane, F, lane_outside, b[0]);
        ldk<K, T, MODE>(rowp(r + gr), c_lane, F, lane_outside, b[1]);
        ldk<K, T, MODE>(rowp(r - gr - 1), c_lane, F, lane_outside, b[2]);
        ldk<K, T, MODE>(rowp(r - hr - 1), c_lane, F, lane_outside, b[3]);
        ldk<K, T, MODE>(rowp(r), c_lane, F, lane_outside, b[4]);
    };
    auto general_rows = [&](int r0, int r1) {
        for (int r = r0; r < r1; ++r) {
            T b[5][K];
            Prep pp;
            prep(r, pp);
            issue(r, b);
            accumulate(r, b);
            output_general(r, b[4], pp);
            __builtin_amdgcn_wave_barrier();
        }
    };

    // Interior rows of FAST and EDGE units without the optional outputs
    // (EDGE: lanes outside the map load column 0, weighed by zero): every
    // row of both windows inside the map, so the accumulators take plain adds and
    // subtractions.  Rows come through a buffer resource over the rows this
    // loop touches, with wave-uniform row offsets that advance one row per
    // step and PD rows in flight, and through a per-wave LDS ring (slot of
    // row i = i mod D, kept as running indices):
    //   FULL: one global load per row (lead row r+hr, also written into a
    //         ring of D = 2hr+2 rows, whence rows r+gr, r-gr-1, r-hr-1 and
    //         the cells under test come back);
    //   else: three global loads per row (rows r+hr, r+gr, r-hr-1); row
    //         r+gr also goes into a ring of D = 2gr+2 rows, whence row
    //         r-gr-1 and the cells under test come back.
    // Needs r0 > hr, r1 <= R - hr and the rows' byte span below 2^31.
    auto interior = [&](auto full_tag, int r0, int r1) {
        constexpr bool FULL = decltype(full_tag)::value;
        if (r0 >= r1) return;
        constexpr int PD = FULL ? prefetch_rows_full<K, T>() : prefetch_rows<K, T>();
        constexpr int NL = FULL ? 1 : 3;  // global loads per row
        const int D = FULL ? 2 * hr + 2 : 2 * gr + 2;
        const int hw = FULL ? hr : gr;  // half-width of the rows the ring serves
        const uint32_t ldb = (uint32_t)ld * (uint32_t)sizeof(T);
        const int row_lo = r0 - hr - 1;
        const int row_hi = r1 - 1 + hr;
        // base and extent are wave-uniform: say so, or the compiler wraps
        // every buffer access in a loop over distinct descriptors
        const uint64_t base = (uint64_t)(uintptr_t)(X + (int64_t)row_lo * ld);
        const uint32_t base_lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
        const uint32_t base_hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
        const int extent = (int)__builtin_amdgcn_readfirstlane((uint32_t)(row_hi - row_lo) * ldb +
                                                               (uint32_t)F * (uint32_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rsx = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(uintptr_t)(((uint64_t)base_hi << 32) | base_lo), (short)0, extent, kBufferFlags);
        const uint32_t voff = lane_outside ? 0u : (uint32_t)c_lane * (uint32_t)sizeof(T);  // EDGE: column 0
        uint32_t so_lead = (uint32_t)(r0 + hr - row_lo) * ldb;
        uint32_t so_glead = (uint32_t)(r0 + gr - row_lo) * ldb;
        uint32_t so_lag = 0;
        auto load = [&](T(&b)[NL][K]) {
            ldk_buf<K, T>(rsx, voff, so_lead, b[0]);
            so_lead += ldb;
            if constexpr (!FULL) {
                ldk_buf<K, T>(rsx, voff, so_glead, b[1]);
                ldk_buf<K, T>(rsx, voff, so_lag, b[2]);
                so_glead += ldb;
                so_lag += ldb;
            }
        };
        // a lane's K values of one ring row, moved as 16-byte LDS accesses
        // where K * sizeof(T) is a multiple of 16 (aligned: the ring starts on
        // a 4 KiB boundary), conflict-free at that lane stride
        typedef uint32_t r32x4 __attribute__((ext_vector_type(4)));
        auto ring_put = [&](int slot, const T(&v)[K]) {
            char *p = (char *)(ring + (slot * 64 + lane) * K);
            if constexpr (K * sizeof(T) % 16 == 0) {
#pragma unroll
                for (int q = 0; q < (int)(K * sizeof(T) / 16); ++q) {
                    r32x4 w;
                    __builtin_memcpy(&w, (const char *)v + 16 * q, 16);
                    *(r32x4 *)(p + 16 * q) = w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) ((T *)p)[k] = v[k];
            }
        };
        auto ring_get = [&](int slot, T(&v)[K]) {
            const char *p = (const char *)(ring + (slot * 64 + lane) * K);
            if constexpr (K * sizeof(T) % 16 == 0) {
#pragma unroll
                for (int q = 0; q < (int)(K * sizeof(T) / 16); ++q) {
                    const r32x4 w = *(const r32x4 *)(p + 16 * q);
                    __builtin_memcpy((char *)v + 16 * q, &w, 16);
                }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) v[k] = ((const T *)p)[k];
            }
        };
        {
            int sl = (r0 - hw - 1) % D;
            uint32_t so = (uint32_t)(hr - hw) * ldb;  // row r0-hw-1
            for (int i = 0; i < D - 1; ++i) {         // rows r0-hw-1 .. r0+hw-1
                T v[K];
                ldk_buf<K, T>(rsx, voff, so, v);
                ring_put(sl, v);
                so += ldb;
                sl = sl + 1 == D ? 0 : sl + 1;
            }
        }
        // running slots: rows r+hw (written), r, and for FULL r+gr, r-gr-1
        int s_w = (r0 + hw) % D, s_c = r0 % D, s_g = (r0 + gr) % D, s_gl = (r0 - gr - 1 + D) % D;
        // The mask rows r0..r1-1 through a buffer resource too; a lane
        // without output columns stores past its end, where the store is
        // dropped, so the store needs no branch (and no alignment: the
        // packed store of a lane may straddle dwords)
        const uint64_t mbase = (uint64_t)(uintptr_t)(d.mask + (int64_t)r0 * d.ld_mask);
        const uint32_t mb_lo = __builtin_amdgcn_readfirstlane((uint32_t)mbase);
        const uint32_t mb_hi = __builtin_amdgcn_readfirstlane((uint32_t)(mbase >> 32));
        const int mext = (int)__builtin_amdgcn_readfirstlane((uint32_t)(r1 - 1 - r0) * (uint32_t)d.ld_mask +
                                                             (uint32_t)F);
        const __amdgpu_buffer_rsrc_t rsm = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(uintptr_t)(((uint64_t)mb_hi << 32) | mb_lo), (short)0, mext, kBufferFlags);
        // (EDGE: a lane of a right-aligned last strip may own only its last
        // K - k_own0 columns; it stores those as bytes, the packed store
        // skips it)
        const uint32_t moff = lane_any_out && k_own0 == 0 ? (uint32_t)c_lane : 0x80000000u;
        const bool unit_partial = BM == kEdge && __ballot(lane_any_out && k_own0 > 0) != 0ull;
        const uint32_t mstep_u = __builtin_amdgcn_readfirstlane((uint32_t)d.ld_mask);
        uint32_t so_m = 0;
        auto next = [&](int v) { return v + 1 == D ? 0 : v + 1; };
        auto step = [&](const T(&b)[NL][K]) {
            T gle[K], gla[K], la[K], xc[K];
            const int s_l = next(s_w);  // row r-hw-1 = r+hw+1 mod D
            {
                ring_put(s_w, b[FULL ? 0 : NL - 2]);
                if constexpr (FULL)
                    ring_get(s_l, la);
                else
                    ring_get(s_l, gla);
                ring_get(s_c, xc);
                if constexpr (FULL) {
                    ring_get(s_g, gle);
                    ring_get(s_gl, gla);
                } else {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        gle[k] = b[NL - 2][k];
                        la[k] = b[NL - 1][k];
                    }
                }
            }
            s_w = s_l;
            s_c = next(s_c);
            if constexpr (FULL) {
                s_g = next(s_g);
                s_gl = next(s_gl);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if constexpr (BM == kEdge) {  // lanes outside the map weigh zero
                    Co[k] = __builtin_fma(-lane_w, (double)la[k], __builtin_fma(lane_w, (double)b[0][k], Co[k]));
                    Ci[k] = __builtin_fma(-lane_w, (double)gla[k], __builtin_fma(lane_w, (double)gle[k], Ci[k]));
                } else {
                    Co[k] = (Co[k] + (double)b[0][k]) - (double)la[k];
                    Ci[k] = (Ci[k] + (double)gle[k]) - (double)gla[k];
                }
            }
            publish();
            uint32_t bits[(K + 3) / 4];
            decide_fast(xc, bits);
            if constexpr (K == 2) {
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)bits[0], rsm, moff, so_m, 0);
            } else if constexpr (K == 4) {
                __builtin_amdgcn_raw_buffer_store_b32(bits[0], rsm, moff, so_m, 0);
            } else {
                typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                const u32x2 w = {bits[0], bits[1]};
                __builtin_amdgcn_raw_buffer_store_b64(w, rsm, moff, so_m, 0);
            }
            if (unit_partial) {  // wave-uniform
                const uint32_t pboff = lane_any_out && k_own0 > 0 ? (uint32_t)c_lane : 0x80000000u;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(bits[k / 4] >> (8 * (k % 4))), rsm,
                                                         k >= k_own0 ? pboff + (uint32_t)k : 0x80000000u, so_m, 0);
            }
            so_m += mstep_u;
        };
        T buf[PD][NL][K];
        int r = r0;
        if (r1 - r0 >= PD) {
#pragma unroll
            for (int j = 0; j < PD; ++j) load(buf[j]);
            for (; r + 2 * PD <= r1; r += PD) {
#pragma unroll
                for (int j = 0; j < PD; ++j) {
                    step(buf[j]);
                    load(buf[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < PD; ++j) step(buf[j]);
            r += PD;
        }
        for (; r < r1; ++r) {
            T b[NL][K];
            load(b);
            step(b);
        }
    };
    // Interior rows without the ring (wide guard windows): five loads per row.
    auto pipelined_fast5 = [&](int r0, int r1) {
        if (r0 >= r1) return;
        T A[5][K], B[5][K];
        issue(r0, A);
        int r = r0;
        for (; r + 1 < r1; r += 2) {
            issue(r + 1, B);  // rows are clamped, so issuing past the end is harmless
            accumulate(r, A);
            output_fast(r, A[4]);
            issue(r + 2, A);
            accumulate(r + 1, B);
            output_fast(r + 1, B[4]);
        }
        if (r < r1) {
            accumulate(r, A);
            output_fast(r, A[4]);
        }
    };
    auto pipelined_general = [&](int r0, int r1) {
        if (r0 >= r1) return;
        T A[5][K], B[5][K];
        Prep PA, PB;
        issue(r0, A);
        int r = r0;
        for (; r + 1 < r1; r += 2) {
            prep(r, PA);
            issue(r + 1, B);
            accumulate(r, A);
            output_general(r, A[4], PA);
            prep(r + 1, PB);
            issue(r + 2, A);
            accumulate(r + 1, B);
            output_general(r + 1, B[4], PB);
        }
        if (r < r1) {
            prep(r, PA);
            accumulate(r, A);
            output_general(r, A[4], PA);
        }
    };
    if (BM != kGeneral && !OUT) {
        const bool span_ok = (d.vec_ok & 4) != 0;
        const int ring_rows = ring_bytes / (64 * K * (int)sizeof(T));
        const int r_in0 = min(max(hr + 1, ra), rb);
        const int r_in1 = max(min(R - hr, rb), r_in0);
        general_rows(ra, r_in0);
        if (BM == kFast && span_ok && 2 * hr + 2 <= ring_rows)  // (EDGE: guard ring only, for registers)
            interior(std::true_type(), r_in0, r_in1);
        else if (span_ok && 2 * gr + 2 <= ring_rows)
            interior(std::false_type(), r_in0, r_in1);
        else
            pipelined_fast5(r_in0, r_in1);
        general_rows(r_in1, rb);
    } else {
        pipelined_general(ra, rb);
    }
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// One wave per workgroup; dynamic LDS per wave: the two prefix rows
// (2*K*64 doubles), then the ring of args.ring_rows rows of 64*K values.
// Mode of one work unit (see fused_unit) and its run.
template <int K, typename T, bool OUT>
__device__ __forceinline__ void run_unit(const MapDesc &d, int strip, int rchunk, double *qo, double *qi, void *ring,
                                         int ring_bytes, int lane)
{
    const int F = d.cols, W = 64 * K;
    int cs = strip * d.tw - d.halo_f;
    const bool halo_ok = (d.halo_f % K) == 0;
    // The last strip, if its lanes would straddle column F (F not a multiple
    // of K), is right-aligned instead: its last lanes then end on column
    // F + H - 1, so column F falls on a lane boundary, and since its outputs
    // start within the last tw columns it still reaches back H columns
    // before them.  (Earlier strips that reach past F take the general path.)
    if (halo_ok && strip == d.n_strips - 1 && cs + W > F && F % K != 0 && F + d.halo_f - W >= 0)
        cs = F + d.halo_f - W;
    const bool inside = cs >= 0 && cs + W <= F;
    // EDGE needs lanes wholly inside or outside: columns 0 and F, where they
    // fall inside the strip, on lane boundaries
    const bool left_ok = cs >= 0 || (cs % K) == 0;
    const bool edge_ok = F >= K && ((F - cs) % K == 0 || cs + W <= F) && left_ok;
    T *rg = (T *)ring;
    if (halo_ok && inside) {
        fused_unit<K, T, kFast, OUT>(d, strip, rchunk, cs, qo, qi, rg, ring_bytes, lane);
    } else if (halo_ok && edge_ok) {
        fused_unit<K, T, kEdge, OUT>(d, strip, rchunk, cs, qo, qi, rg, ring_bytes, lane);
    } else {
        fused_unit<K, T, kGeneral, OUT>(d, strip, rchunk, strip * d.tw - d.halo_f, qo, qi, rg, ring_bytes, lane);
    }
}

#ifndef CFAR_WAVES_16B
#define CFAR_WAVES_16B 3
#endif
// Waves per SIMD the register allocation aims at, by bytes per lane and row
// (the LDS of one wave is small, so registers set the occupancy).
template <int KS, typename T, bool OUT>
constexpr int fused_waves()
{
    return KS == 8 ? 1 : sizeof(T) == 4 ? (OUT ? 2 : CFAR_WAVES_16B) : (OUT ? 1 : 2);
}

// One wave per workgroup; dynamic LDS per wave: the two prefix rows
// (2*kmax*64 doubles), then the ring of args.ring_bytes.  KS = 24: each
// unit runs with its map's k (2 or 4); KS = 8: k = 8.
template <int KS, typename T, bool OUT>
__global__ void __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(fused_waves<KS, T, OUT>())))
fused_kernel(FusedArgs args)
{
    constexpr int KM = KS == 8 ? 8 : 4;
    extern __shared__ double fused_lds[];
    const int lane = threadIdx.x & 63;
    double *qo = fused_lds;
    double *qi = fused_lds + KM * 64;
    T *ring = (T *)(fused_lds + 2 * KM * 64);
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = __hip_atomic_fetch_add(args.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u = wave_uniform(u);
        if (u >= args.total_units) break;
        // descriptor and unit tables are wave-uniform: global (scalar) loads
        uint32_t local = u;
        MapDesc d;
        if (args.descs) {
            const uint32_t m = wave_uniform(gbl(args.unit_map)[u]);
            local = u - wave_uniform(gbl(args.unit_base)[m]);
            const CFAR_GLOBAL uint32_t *src = (const CFAR_GLOBAL uint32_t *)gbl(args.descs + m);
            uint32_t w[sizeof(MapDesc) / 4];
#pragma unroll
            for (int i = 0; i < (int)(sizeof(MapDesc) / 4); ++i) w[i] = src[i];
            __builtin_memcpy(&d, w, sizeof(MapDesc));
        } else {
            d = args.single;
        }
        const int strip = (int)(local % (uint32_t)d.n_strips);
        const int rchunk = (int)(local / (uint32_t)d.n_strips);
        if constexpr (KS == 8) {
            run_unit<8, T, OUT>(d, strip, rchunk, qo, qi, ring, args.ring_bytes, lane);
        } else {
            if (d.k_cols == 2)
                run_unit<2, T, OUT>(d, strip, rchunk, qo, qi, ring, args.ring_bytes, lane);
            else
                run_unit<4, T, OUT>(d, strip, rchunk, qo, qi, ring, args.ring_bytes, lane);
        }
    }
}

#define CFAR_FUSED_VARIANTS(X_)                                                                        \
    X_(24, float, false) X_(24, float, true) X_(24, double, false) X_(24, double, true)                 \
    X_(8, float, false) X_(8, float, true) X_(8, double, false) X_(8, double, true)

static const void *fused_fn(int kset, int dtype, bool out)
{
#define CFAR_PICK(K_, T_, O_)                                             \
    if (kset == K_ && dtype == (sizeof(T_) == 4 ? 0 : 1) && out == O_) \
        return (const void *)fused_kernel<K_, T_, O_>;
    CFAR_FUSED_VARIANTS(CFAR_PICK)
#undef CFAR_PICK
    return nullptr;
}

int fused_resident_blocks(int kset, int dtype, bool out, int ring_bytes)
{
    // cache: device x kernel x ring size (in 512-byte steps)
    constexpr int kSteps = 129;
    static int cached[16][8][kSteps] = {{{0}}};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    const int slot = ((kset == 8 ? 1 : 0) * 2 + dtype) * 2 + (out ? 1 : 0);
    const int step = ring_bytes % 512 == 0 && ring_bytes / 512 < kSteps ? ring_bytes / 512 : -1;
    int *c = dev < 16 && step >= 0 ? &cached[dev][slot][step] : nullptr;
    if (c && *c > 0) return *c;
    const void *fn = fused_fn(kset, dtype, out);
    int per_cu = 0, cus = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kFusedThreads,
                                                            fused_lds_bytes(kset, ring_bytes)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus < 1) cus = 1;
    if (c) *c = per_cu * cus;
    return per_cu * cus;
}

hipError_t launch_fused(const FusedArgs &args, int kset, int dtype, bool out, hipStream_t stream)
{
    const int resident = fused_resident_blocks(kset, dtype, out, args.ring_bytes);
    uint32_t blocks = args.total_units;
    if (blocks > (uint32_t)resident) blocks = (uint32_t)resident;
    if (blocks == 0) blocks = 1;
    const size_t lds = fused_lds_bytes(kset, args.ring_bytes);
#define CFAR_LAUNCH(K_, T_, O_)                                                                                \
    if (kset == K_ && dtype == (sizeof(T_) == 4 ? 0 : 1) && out == O_) {                                       \
        hipLaunchKernelGGL((fused_kernel<K_, T_, O_>), dim3(blocks), dim3(kFusedThreads), lds, stream, args); \
        return hipGetLastError();                                                                              \
    }
    CFAR_FUSED_VARIANTS(CFAR_LAUNCH)
#undef CFAR_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace cfar
