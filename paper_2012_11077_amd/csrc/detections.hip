// Detection lists and bit-packed masks: what the detector's decisions
// (eq. 1, H1 where CUT > T) hand on to a consumer, in fewer bytes than the
// dense mask.  Both read a mask written by cfar2d / cfar2d_batched on the
// same stream.
//
// Detection list: two passes so the records come out in row-major order of
// the cells, whatever the launch order of the workgroups.
//   det_count: block b covers row b / nbc and kDetCols columns of it (256
//              threads x 16 cells); it writes its number of detections;
//   det_scan:  one workgroup turns the counts into exclusive offsets (int64)
//              and the total;
//   det_write: block b recounts, takes each thread's offset from a block
//              scan, and writes the records below the capacity.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace cfar {

constexpr int kDetCells = 16;                 // consecutive cells per thread
constexpr int kDetCols = 256 * kDetCells;     // columns per block

struct DetArgs {
    const uint8_t *mask;
    const void *x;
    const double *thresh;  // optional
    int64_t ld_mask, ld;
    int64_t rows, cols;
    int64_t nbc;           // blocks per row
    int32_t dtype;
    int32_t vec;           // mask base and ld_mask multiples of 16: whole 16-byte loads
};

// Bits of the nonzero bytes of a 32-bit word (byte k -> bit k).
__device__ __forceinline__ uint32_t nz_bytes(uint32_t w)
{
    return ((w & 0xffu) ? 1u : 0u) | ((w & 0xff00u) ? 2u : 0u) | ((w & 0xff0000u) ? 4u : 0u) |
           ((w & 0xff000000u) ? 8u : 0u);
}

// 16 mask bytes at p (16-byte aligned) as 16 bits.
__device__ __forceinline__ uint32_t nz16(const uint8_t *p)
{
    const uint4 v = *(const uint4 *)p;
    return nz_bytes(v.x) | (nz_bytes(v.y) << 4) | (nz_bytes(v.z) << 8) | (nz_bytes(v.w) << 12);
}

__device__ __forceinline__ int det_cells(const DetArgs &a, int64_t b, int64_t &r, int64_t &c0, uint32_t &bits)
{
    r = b / a.nbc;
    c0 = (b - r * a.nbc) * kDetCols + (int64_t)threadIdx.x * kDetCells;
    bits = 0;
    const uint8_t *row = a.mask + r * a.ld_mask;
    if (a.vec && c0 + kDetCells <= a.cols) {
        bits = nz16(row + c0);
    } else {
#pragma unroll
        for (int u = 0; u < kDetCells; ++u) {
            const int64_t c = c0 + u;
            if (c < a.cols && row[c] != 0) bits |= 1u << u;
        }
    }
    return __builtin_popcount(bits);
}

// Exclusive scan of v over the 256 threads of the block (LDS, two levels).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds, uint32_t *total)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t s = v;  // inclusive scan inside the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(s, d, 64);
        if (lane >= d) s += o;
    }
    if (lane == 63) lds[w] = s;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        base += k < w ? lds[k] : 0u;
        tot += lds[k];
    }
    *total = tot;
    return base + s - v;
}

__global__ void __launch_bounds__(256) det_count(DetArgs a, uint32_t *__restrict__ counts)
{
    __shared__ uint32_t lds[4];
    int64_t r, c0;
    uint32_t bits;
    const uint32_t n = (uint32_t)det_cells(a, blockIdx.x, r, c0, bits);
    uint32_t tot;
    block_excl_scan(n, lds, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) det_scan(const uint32_t *__restrict__ counts, int64_t nb,
                                                 int64_t *__restrict__ offsets, int64_t *__restrict__ total)
{
    // four consecutive counts per thread, 4096 per pass
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 4096) {
        const int64_t i0 = base + 4 * (int64_t)t;
        int64_t c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = i0 + q < nb ? (int64_t)counts[i0 + q] : 0;
        const int64_t v = (c[0] + c[1]) + (c[2] + c[3]);
        int64_t s = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t o = __shfl_up(s, d, 64);
            if (lane >= d) s += o;
        }
        if (lane == 63) wsum[w] = s;
        __syncthreads();
        int64_t before = carry;
        int64_t chunk = 0;
        for (int k = 0; k < 16; ++k) {
            before += k < w ? wsum[k] : 0;
            chunk += wsum[k];
        }
        int64_t off = before + s - v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (i0 + q < nb) offsets[i0 + q] = off;
            off += c[q];
        }
        __syncthreads();  // every thread has read carry and wsum
        if (t == 0) carry += chunk;
        __syncthreads();
    }
    if (t == 0) *total = carry;
}

template <typename T>
__global__ void __launch_bounds__(256) det_write(DetArgs a, const int64_t *__restrict__ offsets,
                                                 cfar_detection *__restrict__ out, int64_t capacity)
{
    __shared__ uint32_t lds[4];
    int64_t r, c0;
    uint32_t bits;
    const uint32_t n = (uint32_t)det_cells(a, blockIdx.x, r, c0, bits);
    uint32_t tot;
    int64_t idx = offsets[blockIdx.x] + block_excl_scan(n, lds, &tot);
    const T *x = (const T *)a.x + r * a.ld;
    while (bits) {
        const int u = __builtin_ctz(bits);
        bits &= bits - 1;
        if (idx < capacity) {
            const int64_t c = c0 + u;
            cfar_detection d;
            d.row = (int32_t)r;
            d.col = (int32_t)c;
            d.cut = (double)x[c];
            d.threshold = a.thresh ? a.thresh[r * a.ld_mask + c] : __builtin_nan("");
            out[idx] = d;
        }
        ++idx;
    }
}

// Bit-packed mask: thread per 32-bit word; bit u of word w of row r is cell
// (r, 32 w + u); bits past the last column are 0.
__global__ void __launch_bounds__(256) det_pack(const uint8_t *__restrict__ mask, int64_t ld_mask, int64_t rows,
                                                int64_t cols, int64_t words, uint32_t *__restrict__ bits,
                                                int64_t ld_words, int vec)
{
    const int64_t n = rows * words;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / words, w = i - r * words;
        const uint8_t *row = mask + r * ld_mask + w * 32;
        uint32_t v = 0;
        if (vec && w * 32 + 32 <= cols) {
            v = nz16(row) | (nz16(row + 16) << 16);
        } else {
            const int m = (int)min<int64_t>(32, cols - w * 32);
            for (int u = 0; u < m; ++u) v |= (row[u] != 0 ? 1u : 0u) << u;
        }
        bits[r * ld_words + w] = v;
    }
}

static int mask_vec16(const cfar_map *m) { return ((uintptr_t)m->mask % 16 == 0 && m->ld_mask % 16 == 0) ? 1 : 0; }

static int check_mask_map(const cfar_map *m)
{
    if (!m) return set_error(CFAR_EINVAL, "map is NULL");
    if (m->dtype != CFAR_F32 && m->dtype != CFAR_F64) return set_error(CFAR_EINVAL, "unknown dtype %d", m->dtype);
    if (m->rows < 1 || m->cols < 1 || m->rows > (int64_t(1) << 30) || m->cols > (int64_t(1) << 30))
        return set_error(CFAR_EINVAL, "rows and cols must lie in [1, 2^30]");
    if (m->ld < m->cols || m->ld_mask < m->cols) return set_error(CFAR_EINVAL, "ld or ld_mask < cols");
    if (!m->x || !m->mask) return set_error(CFAR_EINVAL, "x or mask is NULL");
    return CFAR_OK;
}

static int64_t det_blocks(const cfar_map *m) { return m->rows * ((m->cols + kDetCols - 1) / kDetCols); }

}  // namespace cfar

using namespace cfar;

extern "C" {

size_t cfar_detections_workspace_bytes(const cfar_map *m)
{
    if (check_mask_map(m) != CFAR_OK) return 0;
    const int64_t nb = det_blocks(m);
    return align_up((size_t)nb * 4, 256) + align_up((size_t)nb * 8, 256);
}

int cfar_detections(const cfar_map *m, cfar_detection *out, int64_t capacity, int64_t *count, void *ws,
                    size_t ws_bytes, void *stream)
{
    int rc = check_mask_map(m);
    if (rc != CFAR_OK) return rc;
    if (capacity < 0 || (capacity > 0 && !out)) return set_error(CFAR_EINVAL, "capacity < 0, or out is NULL");
    if (!count || !ws) return set_error(CFAR_EINVAL, "count or ws is NULL");
    const int64_t nb = det_blocks(m);
    if (nb > INT32_MAX) return set_error(CFAR_EINVAL, "map too large for the detection list (2^31 blocks)");
    const size_t need = cfar_detections_workspace_bytes(m);
    if (ws_bytes < need) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, need);
    uint32_t *counts = (uint32_t *)ws;
    int64_t *offsets = (int64_t *)((char *)ws + align_up((size_t)nb * 4, 256));
    DetArgs a;
    a.mask = m->mask;
    a.x = m->x;
    a.thresh = m->threshold;
    a.ld_mask = m->ld_mask;
    a.ld = m->ld;
    a.rows = m->rows;
    a.cols = m->cols;
    a.nbc = (m->cols + kDetCols - 1) / kDetCols;
    a.dtype = m->dtype;
    a.vec = mask_vec16(m);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(det_count, dim3((unsigned)nb), dim3(256), 0, s, a, counts);
    hipLaunchKernelGGL(det_scan, dim3(1), dim3(1024), 0, s, (const uint32_t *)counts, nb, offsets, count);
    if (m->dtype == CFAR_F32)
        hipLaunchKernelGGL(det_write<float>, dim3((unsigned)nb), dim3(256), 0, s, a, (const int64_t *)offsets, out,
                           capacity);
    else
        hipLaunchKernelGGL(det_write<double>, dim3((unsigned)nb), dim3(256), 0, s, a, (const int64_t *)offsets,
                           out, capacity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "launch(detections)");
    return CFAR_OK;
}

int cfar_mask_pack(const cfar_map *m, uint32_t *bits, int64_t ld_words, void *stream)
{
    int rc = check_mask_map(m);
    if (rc != CFAR_OK) return rc;
    const int64_t words = (m->cols + 31) / 32;
    if (!bits) return set_error(CFAR_EINVAL, "bits is NULL");
    if (ld_words < words) return set_error(CFAR_EINVAL, "ld_words < ceil(cols / 32)");
    const int64_t n = m->rows * words;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(det_pack, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint8_t *)m->mask,
                       m->ld_mask, m->rows, m->cols, words, bits, ld_words, mask_vec16(m));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "launch(det_pack)");
    return CFAR_OK;
}

}  // extern "C"
