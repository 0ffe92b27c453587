// Internal declarations shared by the host code and the HIP kernels of
// libcfar2d.so.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "cfar2d.h"

#include <cstddef>
#include <cstdint>

namespace cfar {

// ---------------------------------------------------------------------------
// One map as the device sees it.  Built on the host from a cfar_map plus the
// tile plan; 128 bytes so an array of them packs on 128-byte boundaries.
// ---------------------------------------------------------------------------
struct MapDesc {
    const void *x;        // map, rows x cols, leading dimension ld
    uint8_t *mask;        // rows x cols, leading dimension ld_mask
    double *train_sum;    // optional
    double *thresh;       // optional
    double *lut;          // lut[n] = expm1(-ln(pfa)/n) = alpha(n)/n for n = 1..n_full
    int64_t ld;
    int64_t ld_mask;
    double neg_log_pfa;   // -ln(pfa)
    int32_t rows, cols;
    int32_t gr, gf;       // guard half-widths
    int32_t hr, hf;       // outer half-widths (guard + train)
    int32_t dtype;        // 0 = f32, 1 = f64
    int32_t k_cols;       // TILED: columns per lane (2, 4, 8)
    int32_t rs;           // TILED: output rows per work unit
    int32_t halo_f;       // TILED: column halo, >= hf + 1, multiple of 4
    int32_t tw;           // TILED: output columns per strip = 64*k_cols - 2*halo_f
    int32_t n_strips;     // TILED: strips across the columns
    int32_t n_rchunks;    // TILED: row chunks
    int32_t n_full;       // training cells of an unclipped window
    int32_t vec_ok;       // bits: 2 mask rows 4-byte aligned, 4 unit row span < 2^31 bytes (bit 1 unused)
    int32_t pad0;
};
static_assert(sizeof(MapDesc) == 128, "MapDesc must stay 128 bytes");

// Arguments of the persistent TILED kernel.  When descs == nullptr the kernel
// works on the single map in `single` (no device-side descriptor table).
struct FusedArgs {
    const MapDesc *descs;      // n_maps descriptors in device memory, or nullptr
    const uint32_t *unit_map;  // map index of every work unit (device), or nullptr
    const uint32_t *unit_base; // first work unit of every map (device), or nullptr
    uint32_t *counter;         // work counter (device), zeroed by the table kernel
    uint32_t total_units;
    uint32_t n_maps;
    int32_t ring_bytes;        // LDS bytes per wave for the row ring (see ring_rows_cap)
    int32_t pad;
    MapDesc single;
};

// One map of the PLAIN form (integral image in FP64, then the stencil).
struct PlainDesc {
    MapDesc m;            // map, mask, optional outputs, threshold table, window
    double *S;            // rows x cols integral image, leading dimension cols
    double *left;         // [n_strips][rows]: row totals per strip, then the sums left of each strip
    double *V;            // [n_chunks][cols]: strip prefix of chunk column totals, then the sums above
    int32_t n_strips;     // integral image: strips of kPlainW columns
    int32_t n_chunks;     // integral image: chunks of `chunk` rows
    int32_t chunk;
    int32_t st_k;         // stencil: columns per lane (4 or 8; 0: the map takes the per-cell stencil)
    int32_t st_halo;      // stencil: column halo, >= hf + 1, multiple of max(4, st_k)
    int32_t st_tw;        // stencil: output columns per strip = 64*st_k - 2*st_halo
    int32_t st_strips;    // stencil strips
    int32_t st_band;      // stencil: output rows per work unit
    int32_t st_bands;     // stencil bands
    int32_t st_xcd;       // stencil: strips per XCD group (0: units in plain band-major order)
    int32_t pad[16];
};
static_assert(sizeof(PlainDesc) == 256, "PlainDesc must stay 256 bytes");

constexpr int kPlainK = 4;              // integral image: columns per lane
constexpr int kPlainW = 64 * kPlainK;   // integral image: strip width

// Arguments of the PLAIN kernels.  descs == nullptr: the one map in `single`.
struct PlainArgs {
    const PlainDesc *descs;     // n_maps descriptors (device), or nullptr
    const uint32_t *sat_base;   // [n_maps + 1] first integral-image unit of every map (device)
    const uint32_t *st_base;    // [n_maps + 1] first stencil unit of every map (device)
    const uint32_t *blk_base;   // [n_maps + 1] first carry workgroup of every map (device)
    uint32_t n_maps;
    uint32_t sat_units, st_units, carry_blocks;
    PlainDesc single;
};

// Layout of the TILED batch workspace.  The host writes the first part
// (header + descriptors + unit tables) with one host-to-device copy; the
// threshold tables that follow are filled on the device.
struct BatchHeader {
    uint32_t counter[16];  // one work counter per kernel class (wide ring, k set, dtype, outputs)
    uint32_t n_maps;
    uint32_t total_units;
    uint32_t pad[46];
};
static_assert(sizeof(BatchHeader) == 256, "BatchHeader must stay 256 bytes");

// SAT tile geometry of the PLAIN form: 32 rows x 256 columns per workgroup.
constexpr int kSatTH = 32;
constexpr int kSatTW = 256;
// Line spacing of the TILED sat2d layout (FP32 local tiles of 32 x 32).
constexpr int kLine = 32;

// Work areas of sat2d inside its workspace (element offsets computed by
// sat_ws_layout on the host).
struct SatWs {
    double *agg_row;   // [nI][nJ][32]  row sums of every tile
    double *agg_cs;    // [nI][nJ][256] local integral image, last row, of every tile
    double *agg_tot;   // [nI][nJ]      tile totals
    double *left;      // [nI][nJ][32]  sum of X left of the tile, per row
    double *rt;        // [nI][nJ]      sum of tile totals left of the tile (same tile row)
    double *top;       // [nI][nJ][256] S(r0 - 1, j) above the tile
    int64_t nI, nJ;
};

size_t sat_ws_bytes(int64_t rows, int64_t cols);
SatWs sat_ws_layout(void *ws, int64_t rows, int64_t cols);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Host-side helpers shared by the library's translation units.
int set_error(int code, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int validate_map(const cfar_map *m, int idx, int form);
void drop_batch_ctx(hipStream_t s, void *ws);
// One map in the TILED form on a caller-given workspace of
// tiled_single_ws_bytes(m) bytes (m already validated).
int tiled_single_ws(const cfar_map *m, void *ws, size_t ws_bytes, hipStream_t stream);
size_t tiled_single_ws_bytes(const cfar_map *m);

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
// ---------------------------------------------------------------------------

// PLAIN / TILED integral image.  out_form 0: FP64 SAT at `sat` (ld = cols).
// out_form 1: TILED layout at `sat` (see cfar2d.h).
hipError_t launch_sat2d(const void *x, int dtype, int64_t rows, int64_t cols, int64_t ld,
                        int out_form, void *sat, const SatWs &ws, hipStream_t stream);

// Threshold tables (and the work counters) for `n` maps.  descs: device
// table of descriptors that start with a MapDesc, `stride` bytes apart, or
// nullptr with `single` used instead.
hipError_t launch_lut(const void *descs, size_t stride, const MapDesc &single, int n, uint32_t *counter,
                      hipStream_t stream);

// Eight-corner stencil over the PLAIN FP64 SAT of one map.
hipError_t launch_stencil_plain(const MapDesc &d, const double *sat, hipStream_t stream);

// PLAIN form (plain.hip): integral image (aggregate, carry, finalize) and
// the stencil, each one launch over the units of every map in `a`.
// with_stencil = false stops after the integral image (sat2d).  Maps whose
// st_k is 0 get no stencil units (the caller runs launch_stencil_plain).
hipError_t launch_plain(const PlainArgs &a, int dtype_mask, bool with_stencil, bool any_out, hipStream_t stream);

// DIRECT form: output tile of one workgroup (rows x columns) and its LDS.
constexpr int kDirTH = 4, kDirTW = 64;
constexpr size_t kDirMaxLds = 65536;
size_t direct_lds_bytes(int hr, int hf, int dtype);
hipError_t launch_stencil_direct(const MapDesc &d, hipStream_t stream);

// Persistent TILED kernel over all work units in `args`.  One kernel per
// (k set, dtype, out): kset 24 serves maps planned with k = 2 or 4 (one
// launch for both), kset 8 maps with k = 8; out = maps may carry the
// optional training-sum / threshold outputs.
hipError_t launch_fused(const FusedArgs &args, int kset, int dtype, bool out, hipStream_t stream);

// Number of persistent workgroups of that kernel that fit the device.
int fused_resident_blocks(int kset, int dtype, bool out, int ring_bytes);

constexpr int kFusedThreads = 64;  // one wave per workgroup: LDS is sized per wave
constexpr int kMaxK = 8;
constexpr int kMaxRingRows = 64;
constexpr int kDefaultRingBytes = 12288;
constexpr int kRingStretchBytes = 20480;  // largest guard ring given beyond the plan's budget
constexpr int kDefaultMinUnits = 128;
constexpr int kBatchFullUnits = 8192;  // batched work units that fill the chip several times over

inline int kset_of(int k) { return k == 8 ? 8 : 24; }
inline int kmax_of(int kset) { return kset == 8 ? 8 : 4; }

// Rows of 64*k values a ring of `ring_bytes` holds (at most kMaxRingRows).
inline int ring_rows_cap(int k, int dtype, int ring_bytes)
{
    const int cap = ring_bytes / (64 * k * (dtype == 0 ? 4 : 8));
    return cap < kMaxRingRows ? cap : kMaxRingRows;
}

// Ring bytes one map needs under a budget: the guard rows (2*gr+2 rows of
// the strip; three global loads per row step instead of five) if they fit,
// else none.
inline int ring_bytes_needed(int k, int dtype, int hr, int gr, int budget)
{
    (void)hr;
    const int row = 64 * k * (dtype == 0 ? 4 : 8);
    return 2 * gr + 2 <= ring_rows_cap(k, dtype, budget) ? (2 * gr + 2) * row : 0;
}

// Dynamic LDS of one wave of the TILED kernel: the outer and the guard
// prefix row, 64*kmax doubles each, then the guard ring of the launch.
inline size_t fused_lds_bytes(int kset, int ring_bytes)
{
    return (size_t)2 * kmax_of(kset) * 64 * 8 + (size_t)ring_bytes;
}

}  // namespace cfar
