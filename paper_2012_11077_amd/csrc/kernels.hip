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
//       in two separable steps: FP64 column prefix sums give the four row
//       corners as differences of running sums (lead/lag accumulators), a
//       wave-wide FP64 row prefix of those column window sums gives the four
//       column corners as differences read back from LDS.  The integral image
//       itself is never written; one pass over X.
#include "internal.h"

#include <cmath>

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
// TILED form: persistent fused kernel, one instantiation per (K, T).
//
// One wave owns a work unit: a strip of W = 64*K map columns (the strip's
// output columns plus a halo of H >= hf + 1 columns on each side; lane l
// holds columns l*K .. l*K+K-1 of the strip) and rs output rows.  Per output
// row r:
//   1. four FP64 running column sums of the strip, started at row ra - hr,
//      advanced to rows r+hr, r+gr, r-gr-1, r-hr-1 (lead/lag accumulators
//      that add the same rows in the same order, so each lag equals the lead
//      of an earlier step): their differences are the column sums of the
//      outer and inner windows, i.e. the row corners of eq. (4);
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
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ const CFAR_GLOBAL T *gbl(const T *p) { return (const CFAR_GLOBAL T *)p; }
template <typename T>
__device__ __forceinline__ CFAR_GLOBAL T *gbl_w(T *p) { return (CFAR_GLOBAL T *)p; }

// Loads of K consecutive values of one row (row: wave-uniform byte pointer)
// starting at strip column c.  FAST: the K columns lie inside the map and the
// access is 16-byte aligned (vector loads).  !FAST: each column is clamped
// into [0, F) and the value zeroed outside, so every access stays in bounds.
template <int K, typename T, bool FAST>
__device__ __forceinline__ void ldk(const CFAR_GLOBAL char *row, int c, int F, T (&v)[K])
{
    if constexpr (FAST) {
        const uint32_t off = (uint32_t)c * (uint32_t)sizeof(T);
        if constexpr (sizeof(T) == 4) {
            if constexpr (K == 2) {
                const f32x2 f = *(const CFAR_GLOBAL f32x2 *)(row + off);
                v[0] = f.x; v[1] = f.y;
            } else {
#pragma unroll
                for (int q = 0; q < K / 4; ++q) {
                    const f32x4 f = *(const CFAR_GLOBAL f32x4 *)(row + off + 16u * q);
                    v[4 * q + 0] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < K / 2; ++q) {
                const f64x2 f = *(const CFAR_GLOBAL f64x2 *)(row + off + 16u * q);
                v[2 * q + 0] = f.x; v[2 * q + 1] = f.y;
            }
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

// acc += s * v with s = 1.0 (row inside the map) or 0.0 (outside): a
// branch-free add that is bit-identical to adding or skipping the row.
template <int K, typename T>
__device__ __forceinline__ void acc_row(double (&a)[K], const T (&v)[K], double s)
{
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = __builtin_fma(s, (double)v[k], a[k]);
}

// Lane-major LDS layout of one prefix row: position p = l*K + k at
// [k*64 + l].  Rows K .. 2K-2 repeat rows 0 .. K-2 shifted down one lane
// ([(K+k)*64 + l] holds element k of lane l+1).  Reading position p + o for
// element k of every lane, with o = q*K + s (0 <= s < K), is then one load
// at [(k+s)*64 + l+q] for every k: no per-element address select.  Lane
// indices wrap inside the row so every address stays in the wave's region
// (wrapped values only reach positions that are not outputs).
template <int K>
struct OffsetRead {
    int base;
    __device__ __forceinline__ void init(int o, int lane)
    {
        const int q = o >= 0 ? o / K : -((-o + K - 1) / K);
        const int s = o - q * K;
        base = s * 64 + ((lane + q) & 63);
    }
    __device__ __forceinline__ double get(const double *__restrict__ q, int k) const { return q[base + k * 64]; }
};
constexpr int q_rows(int K) { return 2 * K - 1; }

// FAST: every lane's K columns lie inside the map, the map and mask rows are
// aligned for vector access, the strip's output columns are at least hf away
// from both map borders (so only rows can be clipped), and lanes hold either
// K output columns or none.  Otherwise the general path.
//
// Interior rows of FAST units run in a straight-line loop (no branches, no
// optional stores) with the next row's loads in flight, so the compiler's
// memory waits stay exact; border rows and general units run a plain loop.
template <int K, typename T, bool FAST, bool OUT>
__device__ void fused_unit(const MapDesc &d, int strip, int rchunk, double *__restrict__ qo,
                           double *__restrict__ qi, int lane, uint32_t *__restrict__ sink)
{
    const int R = d.rows, F = d.cols;
    const int hr = d.hr, hf = d.hf, gr = d.gr, gf = d.gf;
    const int H = d.halo_f;
    const int c_out0 = strip * d.tw;
    const int c_out1 = min(c_out0 + d.tw, F);
    const int cs = c_out0 - H;  // map column of strip position 0
    const int ra = rchunk * d.rs;
    const int rb = min(ra + d.rs, R);
    const int c_lane = cs + lane * K;
    const T *__restrict__ X = (const T *)d.x;
    const int64_t ld = d.ld;
    const int lo_row = max(0, ra - hr);  // first row any accumulator adds

    const bool lane_any_out = (c_lane + K > c_out0) && (c_lane < c_out1);
    const bool lane_col_interior = (c_lane >= hf) && (c_lane + K - 1 + hf < F);
    const double beta_full = gbl(d.lut)[d.n_full];

    OffsetRead<K> rd_oh, rd_ol, rd_ih, rd_il;
    rd_oh.init(hf, lane);
    rd_ol.init(-hf - 1, lane);
    rd_ih.init(gf, lane);
    rd_il.init(-gf - 1, lane);

    auto rowp = [&](int i) -> const CFAR_GLOBAL char * {
        const int ic = min(max(i, 0), R - 1);
        return (const CFAR_GLOBAL char *)gbl(X + (int64_t)ic * ld);
    };

    double Cl[K], Cg1[K], Cg0[K], Ch0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { Cl[k] = 0.0; Cg1[k] = 0.0; Cg0[k] = 0.0; Ch0[k] = 0.0; }

    // Warm-up: C over rows [ra - hr, ra + hr - 1], snapshots at ra-gr-2 and
    // ra+gr-1; four rows' loads in flight at a time.
    const int e = ra + hr;
    for (int i0 = ra - hr; i0 < e; i0 += 4) {
        T w0[K], w1[K], w2[K], w3[K];
        ldk<K, T, FAST>(rowp(i0 + 0), c_lane, F, w0);
        ldk<K, T, FAST>(rowp(i0 + 1), c_lane, F, w1);
        ldk<K, T, FAST>(rowp(i0 + 2), c_lane, F, w2);
        ldk<K, T, FAST>(rowp(i0 + 3), c_lane, F, w3);
#define CFAR_WARM(J, WV)                                                                    \
    {                                                                                       \
        const int i = i0 + J;                                                               \
        acc_row<K, T>(Cl, WV, (i >= 0 && i < R && i < e) ? 1.0 : 0.0);                    \
        if (i == ra - gr - 2) {                                                             \
            _Pragma("unroll") for (int k = 0; k < K; ++k) Cg0[k] = Cl[k];                   \
        }                                                                                   \
        if (i == ra + gr - 1) {                                                             \
            _Pragma("unroll") for (int k = 0; k < K; ++k) Cg1[k] = Cl[k];                   \
        }                                                                                   \
    }
        CFAR_WARM(0, w0)
        CFAR_WARM(1, w1)
        CFAR_WARM(2, w2)
        CFAR_WARM(3, w3)
#undef CFAR_WARM
    }

    const int lane_dn = (lane + 63) & 63;
    // Advance the column prefix sums to rows r+hr, r+gr, r-gr-1, r-hr-1; form
    // the column window sums (row corners of eq. 4); prefix them across the
    // strip and publish the prefixes in LDS.
    auto accumulate = [&](int r, const T(&b)[5][K]) {
        acc_row<K, T>(Cl, b[0], r + hr < R ? 1.0 : 0.0);
        acc_row<K, T>(Cg1, b[1], r + gr < R ? 1.0 : 0.0);
        acc_row<K, T>(Cg0, b[2], r - gr - 1 >= lo_row ? 1.0 : 0.0);
        acc_row<K, T>(Ch0, b[3], r - hr - 1 >= lo_row ? 1.0 : 0.0);
        double po[K], pi[K];
        po[0] = Cl[0] - Ch0[0];
        pi[0] = Cg1[0] - Cg0[0];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            po[k] = po[k - 1] + (Cl[k] - Ch0[k]);
            pi[k] = pi[k - 1] + (Cg1[k] - Cg0[k]);
        }
        const double eo = wave_shift_up1(wave_incl_scan(po[K - 1]));
        const double ei = wave_shift_up1(wave_incl_scan(pi[K - 1]));
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double vo = eo + po[k], vi = ei + pi[k];
            qo[k * 64 + lane] = vo;
            qi[k * 64 + lane] = vi;
            if (k < K - 1) {
                qo[(K + k) * 64 + lane_dn] = vo;
                qi[(K + k) * 64 + lane_dn] = vi;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto train_sum_at = [&](int k) -> double {
        // column corners of eq. (4): box = Q(p + h) - Q(p - h - 1), outer minus inner
        return (rd_oh.get(qo, k) - rd_ol.get(qo, k)) - (rd_ih.get(qi, k) - rd_il.get(qi, k));
    };
    CFAR_GLOBAL uint8_t *sink_b = (CFAR_GLOBAL uint8_t *)gbl_w(sink + lane * 2);
    // Interior row of a FAST unit: N = n_full, beta = beta_full, every lane
    // computes; lanes without outputs store into the sink.
    auto output_fast = [&](int r, const T(&xcut)[K]) {
        uint32_t bits[(K + 3) / 4];
#pragma unroll
        for (int q = 0; q < (K + 3) / 4; ++q) bits[q] = 0u;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double thr = beta_full * train_sum_at(k);
            bits[k / 4] |= ((double)xcut[k] > thr) ? (1u << (8 * (k % 4))) : 0u;
        }
        CFAR_GLOBAL uint8_t *mdst = gbl_w(d.mask) + (int64_t)r * d.ld_mask + c_lane;
        CFAR_GLOBAL uint8_t *dst = lane_any_out ? mdst : sink_b;
        if constexpr (K == 2) {
            __builtin_nontemporal_store((uint16_t)bits[0], (CFAR_GLOBAL uint16_t *)dst);
        } else {
#pragma unroll
            for (int q = 0; q < K / 4; ++q) __builtin_nontemporal_store(bits[q], (CFAR_GLOBAL uint32_t *)dst + q);
        }
    };
    // Any row: N and beta per cell.  Branch-free: every cell is computed and
    // its byte stored either into the mask or, outside this strip's outputs,
    // into the sink.  The per-cell table loads are issued by prep() before the
    // next row's loads, so waiting for them never waits for the prefetch.
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
            CFAR_GLOBAL uint8_t *dst = own ? mrow + j : sink_b + k;
            *dst = (uint8_t)(pp.nt[k] > 0 && (double)xcut[k] > thr);
            if constexpr (OUT) {
                if (own) {
                    if (d.train_sum) gbl_w(d.train_sum)[orow + j] = st;
                    if (d.thresh) gbl_w(d.thresh)[orow + j] = pp.nt[k] > 0 ? thr : INFINITY;
                }
            }
        }
    };
    auto issue = [&](int r, T(&b)[5][K]) {
        ldk<K, T, FAST>(rowp(r + hr), c_lane, F, b[0]);
        ldk<K, T, FAST>(rowp(r + gr), c_lane, F, b[1]);
        ldk<K, T, FAST>(rowp(r - gr - 1), c_lane, F, b[2]);
        ldk<K, T, FAST>(rowp(r - hr - 1), c_lane, F, b[3]);
        ldk<K, T, FAST>(rowp(r), c_lane, F, b[4]);
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
    // Rows with the next row's loads in flight (two alternating buffers).
    // FAST units without the optional outputs take the straight-line output
    // on interior rows; all other rows take the general output.
    auto pipelined_fast = [&](int r0, int r1) {
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
    if (FAST && !OUT) {
        const int r_in0 = min(max(hr, ra), rb);
        const int r_in1 = max(min(R - hr, rb), r_in0);
        general_rows(ra, r_in0);
        pipelined_fast(r_in0, r_in1);
        general_rows(r_in1, rb);
    } else {
        pipelined_general(ra, rb);
    }
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }



template <int K, typename T, bool OUT>
__global__ void __launch_bounds__(kFusedThreads) fused_kernel(FusedArgs args)
{
    __shared__ double qbuf[kFusedThreads / 64][2][q_rows(K) * 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    double *qo = qbuf[wave][0];
    double *qi = qbuf[wave][1];
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
        const int cs = strip * d.tw - d.halo_f;
        const bool fast = d.vec_ok == 3 && cs >= 0 && cs + 64 * K <= d.cols && (d.halo_f % K) == 0;
        if (fast)
            fused_unit<K, T, true, OUT>(d, strip, rchunk, qo, qi, lane, args.sink);
        else
            fused_unit<K, T, false, OUT>(d, strip, rchunk, qo, qi, lane, args.sink);
    }
}

#define CFAR_FUSED_VARIANTS(X_)                                                                          \
    X_(2, float, false) X_(4, float, false) X_(8, float, false) X_(2, double, false) X_(4, double, false) \
    X_(8, double, false) X_(2, float, true) X_(4, float, true) X_(8, float, true) X_(2, double, true)     \
    X_(4, double, true) X_(8, double, true)

static const void *fused_fn(int k, int dtype, bool out)
{
#define CFAR_PICK(K_, T_, O_) \
    if (k == K_ && dtype == (sizeof(T_) == 4 ? 0 : 1) && out == O_) return (const void *)fused_kernel<K_, T_, O_>;
    CFAR_FUSED_VARIANTS(CFAR_PICK)
#undef CFAR_PICK
    return nullptr;
}

int fused_resident_blocks(int k, int dtype, bool out)
{
    static int cached[64][16] = {{0}};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    const int slot = ((k == 2 ? 0 : k == 4 ? 1 : 2) * 2 + dtype) * 2 + (out ? 1 : 0);
    if (cached[dev][slot] > 0) return cached[dev][slot];
    const void *fn = fused_fn(k, dtype, out);
    int per_cu = 0, cus = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kFusedThreads, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus < 1) cus = 1;
    cached[dev][slot] = per_cu * cus;
    return cached[dev][slot];
}

hipError_t launch_fused(const FusedArgs &args, int k, int dtype, bool out, hipStream_t stream)
{
    const int resident = fused_resident_blocks(k, dtype, out);
    uint32_t blocks = (args.total_units + (kFusedThreads / 64) - 1) / (kFusedThreads / 64);
    if (blocks > (uint32_t)resident) blocks = (uint32_t)resident;
    if (blocks == 0) blocks = 1;
#define CFAR_LAUNCH(K_, T_, O_)                                                                              \
    if (k == K_ && dtype == (sizeof(T_) == 4 ? 0 : 1) && out == O_) {                                        \
        hipLaunchKernelGGL((fused_kernel<K_, T_, O_>), dim3(blocks), dim3(kFusedThreads), 0, stream, args); \
        return hipGetLastError();                                                                            \
    }
    CFAR_FUSED_VARIANTS(CFAR_LAUNCH)
#undef CFAR_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace cfar
