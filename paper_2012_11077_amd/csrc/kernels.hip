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
//       border windows; also zeroes the work counter of the fused kernel.
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
    if (blockIdx.x == 0 && threadIdx.x == 0 && counter) *counter = 0u;
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
// TILED form: persistent fused kernel.
// ---------------------------------------------------------------------------

// Per-wave LDS: two prefix rows (outer, inner) of 64*K + 1 doubles each; the
// first entry of each row is a zero so that an empty prefix needs no branch.
constexpr int kQStride = 64 * kMaxK + 8;

// Load K consecutive values of one row starting at column c (zero outside [0, F)).
template <int K, typename T>
__device__ __forceinline__ void load_k(const T *__restrict__ row, int c, int F, bool full, bool vec, double (&v)[K])
{
    if (full) {
        if constexpr (sizeof(T) == 4) {
            if (vec && (K % 4) == 0) {
#pragma unroll
                for (int q = 0; q < K / 4; ++q) {
                    const float4 f = *((const float4 *)(row + c) + q);
                    v[4 * q + 0] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
                }
                return;
            }
            if (vec && K == 2) {
                const float2 f = *((const float2 *)(row + c));
                v[0] = f.x; v[1] = f.y;
                return;
            }
        } else {
            if (vec && (K % 2) == 0) {
#pragma unroll
                for (int q = 0; q < K / 2; ++q) {
                    const double2 f = *((const double2 *)(row + c) + q);
                    v[2 * q + 0] = f.x; v[2 * q + 1] = f.y;
                }
                return;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (double)row[c + k];
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int cc = c + k;
            v[k] = (cc >= 0 && cc < F) ? (double)row[cc] : 0.0;
        }
    }
}

template <int K>
__device__ __forceinline__ void acc_k(double (&a)[K], const double (&v)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] += v[k];
}

template <int K, typename T>
__device__ void fused_unit(const MapDesc &d, int strip, int rchunk, double *__restrict__ qo,
                           double *__restrict__ qi, int lane)
{
    constexpr int W = 64 * K;
    const int R = d.rows, F = d.cols;
    const int hr = d.hr, hf = d.hf, gr = d.gr, gf = d.gf;
    const int H = d.halo_f;
    const int c_out0 = strip * d.tw;
    const int c_out1 = min(c_out0 + d.tw, F);
    const int cs = c_out0 - H;  // map column of position 0 of this strip
    const int ra = rchunk * d.rs;
    const int rb = min(ra + d.rs, R);
    const int c_lane = cs + lane * K;
    const bool full = c_lane >= 0 && c_lane + K <= F;
    const bool vec = (d.vec_ok & 1) != 0;
    const T *__restrict__ X = (const T *)d.x;
    const int64_t ld = d.ld;
    const int lo_row = max(0, ra - hr);  // first row any accumulator may add

    // lane's output positions: p = lane*K + k, column j = cs + p, output iff c_out0 <= j < c_out1
    const bool lane_any_out = (c_lane + K > c_out0) && (c_lane < c_out1);
    const bool lane_all_out = (c_lane >= c_out0) && (c_lane + K <= c_out1);
    const bool lane_col_interior = (c_lane >= hf) && (c_lane + K - 1 + hf < F);
    const double beta_full = d.lut[d.n_full];

    if (lane == 0) { qo[0] = 0.0; qi[0] = 0.0; }

    // Column prefix sums C(i) = sum of X over rows [ra - hr, i] of each lane column.
    double Cl[K], Cg1[K], Cg0[K], Ch0[K], v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { Cl[k] = 0.0; Cg1[k] = 0.0; Cg0[k] = 0.0; Ch0[k] = 0.0; }

    // Warm-up: C up to row ra + hr - 1, snapshots at ra - gr - 2 and ra + gr - 1.
    for (int i = ra - hr; i < ra + hr; ++i) {
        if (i >= 0 && i < R) {
            load_k<K, T>(X + (int64_t)i * ld, c_lane, F, full, vec, v);
            acc_k<K>(Cl, v);
        }
        if (i == ra - gr - 2) {
#pragma unroll
            for (int k = 0; k < K; ++k) Cg0[k] = Cl[k];
        }
        if (i == ra + gr - 1) {
#pragma unroll
            for (int k = 0; k < K; ++k) Cg1[k] = Cl[k];
        }
    }

    const bool vec_mask = ((d.vec_ok & 2) != 0) && lane_all_out;
    for (int r = ra; r < rb; ++r) {
        // advance the four accumulators to C(r+hr), C(r+gr), C(r-gr-1), C(r-hr-1)
        if (r + hr < R) { load_k<K, T>(X + (int64_t)(r + hr) * ld, c_lane, F, full, vec, v); acc_k<K>(Cl, v); }
        if (r + gr < R) { load_k<K, T>(X + (int64_t)(r + gr) * ld, c_lane, F, full, vec, v); acc_k<K>(Cg1, v); }
        if (r - gr - 1 >= lo_row) { load_k<K, T>(X + (int64_t)(r - gr - 1) * ld, c_lane, F, full, vec, v); acc_k<K>(Cg0, v); }
        if (r - hr - 1 >= lo_row) { load_k<K, T>(X + (int64_t)(r - hr - 1) * ld, c_lane, F, full, vec, v); acc_k<K>(Ch0, v); }

        // column window sums (row corners of eq. 4) and their row prefix within the lane
        double po[K], pi[K];
        po[0] = Cl[0] - Ch0[0];
        pi[0] = Cg1[0] - Cg0[0];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            po[k] = po[k - 1] + (Cl[k] - Ch0[k]);
            pi[k] = pi[k - 1] + (Cg1[k] - Cg0[k]);
        }
        // wave-wide exclusive offsets
        const double eo = wave_shift_up1(wave_incl_scan(po[K - 1]));
        const double ei = wave_shift_up1(wave_incl_scan(pi[K - 1]));
#pragma unroll
        for (int k = 0; k < K; ++k) {
            qo[1 + lane * K + k] = eo + po[k];
            qi[1 + lane * K + k] = ei + pi[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        if (lane_any_out) {
            // column corners of eq. (4) from the row prefixes: box = Q(p+h) - Q(p-h-1)
            const bool row_interior = (r >= hr) && (r + hr < R);
            const bool interior = row_interior && lane_col_interior;
            const int nro = clip_len(r, hr, R), nri = clip_len(r, gr, R);
            double cut[K];
            load_k<K, T>(X + (int64_t)r * ld, c_lane, F, full, vec, cut);
            uint8_t m[K];
            const int64_t orow = (int64_t)r * d.ld_mask;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                // positions outside this strip's outputs are evaluated at a clamped
                // position (their results are discarded) so every index stays in bounds
                const int p = min(max(lane * K + k, H), W - H - 1);
                const double bo = qo[p + hf + 1] - qo[p - hf];
                const double bi = qi[p + gf + 1] - qi[p - gf];
                const double st = bo - bi;
                int nt;
                double beta;
                if (interior) {
                    nt = d.n_full;
                    beta = beta_full;
                } else {
                    const int j = min(cs + p, F - 1);
                    nt = nro * clip_len(j, hf, F) - nri * clip_len(j, gf, F);
                    beta = d.lut[nt];
                }
                const double thr = beta * st;
                m[k] = (uint8_t)(nt > 0 && cut[k] > thr);
                if (d.train_sum || d.thresh) {
                    const int j = c_lane + k;
                    if (j >= c_out0 && j < c_out1) {
                        if (d.train_sum) d.train_sum[orow + j] = st;
                        if (d.thresh) d.thresh[orow + j] = nt > 0 ? thr : INFINITY;
                    }
                }
            }
            uint8_t *mrow = d.mask + orow;
            if (vec_mask && (K % 4) == 0) {
#pragma unroll
                for (int q = 0; q < K / 4; ++q) {
                    const uint32_t w = (uint32_t)m[4 * q] | ((uint32_t)m[4 * q + 1] << 8) |
                                       ((uint32_t)m[4 * q + 2] << 16) | ((uint32_t)m[4 * q + 3] << 24);
                    __builtin_nontemporal_store(w, (uint32_t *)(mrow + c_lane) + q);
                }
            } else if (vec_mask && K == 2) {
                const uint16_t w = (uint16_t)((uint32_t)m[0] | ((uint32_t)m[1] << 8));
                __builtin_nontemporal_store(w, (uint16_t *)(mrow + c_lane));
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int j = c_lane + k;
                    if (j >= c_out0 && j < c_out1) mrow[j] = m[k];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ __forceinline__ uint32_t wave_uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ void __launch_bounds__(kFusedThreads) fused_kernel(FusedArgs args)
{
    __shared__ double qbuf[kFusedThreads / 64][2][kQStride];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    double *qo = qbuf[wave][0];
    double *qi = qbuf[wave][1];
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = atomicAdd(args.counter, 1u);
        u = wave_uniform(u);
        if (u >= args.total_units) break;
        const MapDesc *dp;
        uint32_t local;
        if (args.descs) {
            const uint32_t m = wave_uniform(args.unit_map[u]);
            dp = args.descs + m;
            local = u - wave_uniform(args.unit_base[m]);
        } else {
            dp = &args.single;
            local = u;
        }
        const MapDesc d = *dp;
        const int strip = (int)(local % (uint32_t)d.n_strips);
        const int rchunk = (int)(local / (uint32_t)d.n_strips);
        const int key = d.k_cols * 2 + d.dtype;
        switch (key) {
        case 2 * 2 + 0: fused_unit<2, float>(d, strip, rchunk, qo, qi, lane); break;
        case 2 * 2 + 1: fused_unit<2, double>(d, strip, rchunk, qo, qi, lane); break;
        case 4 * 2 + 0: fused_unit<4, float>(d, strip, rchunk, qo, qi, lane); break;
        case 4 * 2 + 1: fused_unit<4, double>(d, strip, rchunk, qo, qi, lane); break;
        case 8 * 2 + 0: fused_unit<8, float>(d, strip, rchunk, qo, qi, lane); break;
        case 8 * 2 + 1: fused_unit<8, double>(d, strip, rchunk, qo, qi, lane); break;
        default: break;
        }
    }
}

hipError_t launch_fused(const FusedArgs &args, hipStream_t stream)
{
    const int resident = fused_resident_blocks();
    const uint32_t waves_needed = args.total_units;
    uint32_t blocks = (waves_needed + (kFusedThreads / 64) - 1) / (kFusedThreads / 64);
    if (blocks > (uint32_t)resident) blocks = (uint32_t)resident;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(fused_kernel, dim3(blocks), dim3(kFusedThreads), 0, stream, args);
    return hipGetLastError();
}

int fused_resident_blocks()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cached[dev] > 0) return cached[dev];
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel, kFusedThreads, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus < 1) cus = 1;
    cached[dev] = per_cu * cus;
    return cached[dev];
}

}  // namespace cfar
