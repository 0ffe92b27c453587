// Host side of libcfar2d.so: argument validation, tile plans, workspace
// layout, launch sequences, hipGraph capture/replay for batches.
//
// Method: arXiv 2012.11077, Sec. II.B (eqs. 1-4); see include/cfar2d.h.
#include "cfar2d.h"
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

namespace cfar {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    return set_error(CFAR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Kernel timing (thread-local): HIP events around the persistent kernel of
// TILED launches that are not captured in a graph.
// ---------------------------------------------------------------------------
struct Timing {
    bool on = false;
    bool recorded = false;
    hipEvent_t start = nullptr, stop = nullptr;
};
static thread_local Timing g_timing;

static hipError_t timing_mark(hipEvent_t ev, hipStream_t stream)
{
    return g_timing.on ? hipEventRecord(ev, stream) : hipSuccess;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
constexpr int64_t kMaxDim = int64_t(1) << 30;  // rows, cols
constexpr int32_t kMaxHalf = 1024;             // any half-width
constexpr int32_t kMaxTiledHf = 247;           // TILED: 64*8 columns per wave minus two halos

// Most output rows one TILED work unit may take: the byte offsets of the
// rows a unit reads (its rows and hr + 1 rows above and below) and of its
// mask rows stay below 2^31.
static int64_t unit_rows_cap(const cfar_map *m)
{
    const int64_t hr = (int64_t)m->win.guard_r + m->win.train_r;
    const int64_t pitch = m->ld * (m->dtype == CFAR_F32 ? 4 : 8);
    const int64_t lim = ((int64_t)1 << 31) - 1;
    return std::min(lim / std::max<int64_t>(pitch, 1) - 2 * hr - 2, lim / std::max<int64_t>(m->ld_mask, 1));
}

int validate_map(const cfar_map *m, int idx, int form)
{
    if (!m) return set_error(CFAR_EINVAL, "map %d: NULL descriptor", idx);
    if (m->reserved0 != 0) return set_error(CFAR_EINVAL, "map %d: reserved0 must be 0", idx);
    if (m->dtype != CFAR_F32 && m->dtype != CFAR_F64)
        return set_error(CFAR_EINVAL, "map %d: unknown dtype %d", idx, m->dtype);
    if (m->rows < 1 || m->cols < 1)
        return set_error(CFAR_EINVAL, "map %d: rows and cols must be >= 1 (got %lld x %lld)", idx,
                         (long long)m->rows, (long long)m->cols);
    if (m->rows > kMaxDim || m->cols > kMaxDim)
        return set_error(CFAR_EINVAL, "map %d: rows and cols must be <= 2^30", idx);
    if (m->ld < m->cols) return set_error(CFAR_EINVAL, "map %d: ld < cols", idx);
    if (m->ld_mask < m->cols) return set_error(CFAR_EINVAL, "map %d: ld_mask < cols", idx);
    if (!m->x) return set_error(CFAR_EINVAL, "map %d: x is NULL", idx);
    if (!m->mask) return set_error(CFAR_EINVAL, "map %d: mask is NULL", idx);
    const cfar_window &w = m->win;
    if (w.guard_r < 0 || w.guard_f < 0 || w.train_r < 0 || w.train_f < 0)
        return set_error(CFAR_EINVAL, "map %d: negative guard or training half-width", idx);
    if (w.train_r + w.train_f == 0) return set_error(CFAR_EINVAL, "map %d: no training cells (train_r + train_f == 0)", idx);
    if ((int64_t)w.guard_r + w.train_r > kMaxHalf || (int64_t)w.guard_f + w.train_f > kMaxHalf)
        return set_error(CFAR_EINVAL, "map %d: guard + train half-width above %d", idx, kMaxHalf);
    if (!(w.pfa > 0.0 && w.pfa < 1.0) || !std::isfinite(w.pfa))
        return set_error(CFAR_EINVAL, "map %d: pfa must lie in (0, 1)", idx);
    if (form != CFAR_FORM_PLAIN && form != CFAR_FORM_TILED && form != CFAR_FORM_DIRECT)
        return set_error(CFAR_EINVAL, "unknown form %d", form);
    if (form == CFAR_FORM_TILED && w.guard_f + w.train_f > kMaxTiledHf)
        return set_error(CFAR_EINVAL, "map %d: TILED form supports guard_f + train_f <= %d (use PLAIN)", idx,
                         kMaxTiledHf);
    if (form == CFAR_FORM_TILED && unit_rows_cap(m) < 1)
        return set_error(CFAR_EINVAL, "map %d: TILED form needs (2 (guard_r + train_r) + 3) rows of the map, and "
                         "one mask row, to span less than 2^31 bytes", idx);
    if (form == CFAR_FORM_DIRECT) {
        if (direct_lds_bytes(w.guard_r + w.train_r, w.guard_f + w.train_f, m->dtype) > kDirMaxLds)
            return set_error(CFAR_EINVAL, "map %d: DIRECT form supports (%d + 2 hr) x (%d + 2 hf) x element size "
                                          "<= %zu bytes (use TILED or PLAIN)", idx, kDirTH, kDirTW, kDirMaxLds);
        const int64_t nb = (m->rows + kDirTH - 1) / kDirTH * ((m->cols + kDirTW - 1) / kDirTW);
        if (nb > INT32_MAX) return set_error(CFAR_EINVAL, "map %d: DIRECT form supports up to 2^31 - 1 tiles", idx);
    }
    return CFAR_OK;
}

static int64_t n_full_of(const cfar_window &w)
{
    const int64_t hr = w.guard_r + w.train_r, hf = w.guard_f + w.train_f;
    return (2 * hr + 1) * (2 * hf + 1) - (int64_t)(2 * w.guard_r + 1) * (2 * w.guard_f + 1);
}

static size_t lut_bytes(const cfar_map *m) { return align_up((size_t)(n_full_of(m->win) + 1) * 8, 256); }

// ---------------------------------------------------------------------------
// Tile plans of the TILED form
// ---------------------------------------------------------------------------
struct Plan {
    int k, rs, H, tw, n_strips, n_rchunks;
    int ring_bytes;  // LDS ring budget per wave (resolved: >= 0)
};

static int ring_budget();
static int min_units();

static bool plan_geometry(const cfar_map *m, int k, int rs, Plan *p, int ring_bytes = -1)
{
    const int hf = m->win.guard_f + m->win.train_f;
    rs = (int)std::min<int64_t>(rs, unit_rows_cap(m));
    // >= hf + 1 (every prefix read stays inside the strip) and a multiple of
    // max(4, k) (lanes hold either k output columns or none)
    const int a = k > 4 ? k : 4;
    const int H = (hf + 1 + a - 1) / a * a;
    const int tw = 64 * k - 2 * H;
    if (tw < 4 || rs < 1) return false;
    p->k = k;
    p->rs = rs;
    p->H = H;
    p->tw = tw;
    p->n_strips = (int)((m->cols + tw - 1) / tw);
    p->n_rchunks = (int)((m->rows + rs - 1) / rs);
    p->ring_bytes = ring_bytes >= 0 ? ring_bytes : ring_budget();
    return true;
}

static uint64_t units_of(const Plan &p) { return (uint64_t)p.n_strips * (uint64_t)p.n_rchunks; }

struct PlanRule {
    int dtype;                    // -1 = any
    int64_t c_lo, c_hi, r_lo, r_hi;
    int hf_lo, hf_hi, hr_lo, hr_hi;
    int k, rs, ring_bytes;
};
static std::mutex g_plan_mu;
static std::vector<PlanRule> g_rules;

// Built-in cost model (fitted to timings of the uneven batch on gfx950): a
// strip row costs c(k) with c(2) = c(4) = 1 (the row step's scans, LDS
// exchange and loop work are per wave, whatever the strip width), c(8) = 3
// (c(2) = 0.9 when k = 2 can hold its guard rows in the LDS ring and k = 4
// cannot); a map narrower than one strip whose last column falls inside a
// lane takes the general path, about three times the cost.  Rows per unit:
// 256 for maps of at least 1024 rows, 64 below (CFAR2D_RS_TALL,
// CFAR2D_RS_SHORT and CFAR2D_COST_K2 override them, for tuning).
static int env_int(const char *name, int dflt)
{
    const char *e = std::getenv(name);
    return e && std::atoi(e) > 0 ? std::atoi(e) : dflt;
}
static int rs_tall()
{
    static const int v = env_int("CFAR2D_RS_TALL", 256);
    return v;
}
static int rs_short()
{
    static const int v = env_int("CFAR2D_RS_SHORT", 64);
    return v;
}
static double cost_k2()
{
    static double v = -1.0;
    if (v < 0.0) {
        const char *e = std::getenv("CFAR2D_COST_K2");
        v = e && std::atof(e) > 0.0 ? std::atof(e) : 1.0;
    }
    return v;
}

static cfar_plan default_plan(const cfar_map *m, bool spread)
{
    const int hr = m->win.guard_r + m->win.train_r;
    static const int ks[3] = {2, 4, 8};
    double best = 1e300;
    int bk = 4;
    for (int t = 0; t < 3; ++t) {
        const int k = ks[t];
        Plan p;
        if (!plan_geometry(m, k, 64, &p)) continue;
        const bool ring2 = 2 * hr + 2 <= ring_rows_cap(2, m->dtype, ring_budget());
        const bool ring4 = 2 * hr + 2 <= ring_rows_cap(4, m->dtype, ring_budget());
        const double c = k == 2 ? (ring2 && !ring4 ? 0.9 : 1.0) * cost_k2() : k == 4 ? 1.0 : 3.0;
        double cost = (double)p.n_strips * c;
        // a map narrower than one strip whose last column falls inside a
        // lane takes the general path
        if (m->cols % k != 0 && m->cols + p.H < 64 * k) cost *= 3.0;
        if (cost < best * 0.999) { best = cost; bk = k; }
    }
    cfar_plan out;
    out.k_cols = bk;
    // tall maps: longer units spread the warm-up rows (2 hr + 1 per unit)
    // over more output rows; the rest keep short units, which also keep the
    // end of a batched launch short (its maps run largest first)
    out.rows_per_unit = (int)std::min<int64_t>(m->rows >= 1024 ? rs_tall() : rs_short(), m->rows);
    // a map of few units runs on few waves, each walking its rows in turn:
    // shorter units (not below 16 rows) spread it over more of the chip
    Plan g;
    if (spread && plan_geometry(m, bk, out.rows_per_unit, &g) && units_of(g) < (uint64_t)min_units()) {
        const int64_t want = (m->rows * g.n_strips + min_units() - 1) / min_units();
        const int64_t rs = std::max<int64_t>(16, (want + 7) / 8 * 8);
        if (rs < out.rows_per_unit) out.rows_per_unit = (int)rs;
    }
    out.ring_bytes = -1;
    return out;
}

// spread: shorten the units of a map of few units (see default_plan); a batch
// with work enough for the chip does without.
static cfar_plan choose_plan(const cfar_map *m, bool spread = true)
{
    const int hr = m->win.guard_r + m->win.train_r, hf = m->win.guard_f + m->win.train_f;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (const PlanRule &r : g_rules) {
            if (r.dtype >= 0 && r.dtype != m->dtype) continue;
            if (m->cols < r.c_lo || m->cols > r.c_hi || m->rows < r.r_lo || m->rows > r.r_hi) continue;
            if (hf < r.hf_lo || hf > r.hf_hi || hr < r.hr_lo || hr > r.hr_hi) continue;
            Plan p;
            if (!plan_geometry(m, r.k, r.rs, &p)) continue;
            cfar_plan out;
            out.k_cols = r.k;
            out.rows_per_unit = (int)std::min<int64_t>(r.rs, m->rows);
            out.ring_bytes = r.ring_bytes;
            return out;
        }
    }
    return default_plan(m, spread);
}

static bool plan_valid(const cfar_map *m, const cfar_plan *p)
{
    if (!(p->k_cols == 2 || p->k_cols == 4 || p->k_cols == 8)) return false;
    if (p->rows_per_unit < 1 || p->rows_per_unit > 4096) return false;
    if (p->ring_bytes < -1 || p->ring_bytes > 65536) return false;
    Plan g;
    return plan_geometry(m, p->k_cols, p->rows_per_unit, &g);
}

// ---------------------------------------------------------------------------
// Descriptors
// ---------------------------------------------------------------------------
static MapDesc make_desc(const cfar_map *m, const Plan *p, double *lut)
{
    MapDesc d;
    std::memset(&d, 0, sizeof d);
    d.x = m->x;
    d.mask = m->mask;
    d.train_sum = m->train_sum;
    d.thresh = m->threshold;
    d.lut = lut;
    d.ld = m->ld;
    d.ld_mask = m->ld_mask;
    d.neg_log_pfa = -std::log(m->win.pfa);
    d.rows = (int32_t)m->rows;
    d.cols = (int32_t)m->cols;
    d.gr = m->win.guard_r;
    d.gf = m->win.guard_f;
    d.hr = m->win.guard_r + m->win.train_r;
    d.hf = m->win.guard_f + m->win.train_f;
    d.dtype = m->dtype;
    d.n_full = (int32_t)n_full_of(m->win);
    if (p) {
        d.k_cols = p->k;
        d.rs = p->rs;
        d.halo_f = p->H;
        d.tw = p->tw;
        d.n_strips = p->n_strips;
        d.n_rchunks = p->n_rchunks;
        const size_t es = m->dtype == CFAR_F32 ? 4 : 8;
        const bool m_vec = ((uintptr_t)m->mask % 4 == 0) && (m->ld_mask % 4 == 0);
        // bit 4: the rows one work unit reads span fewer than 2^31 bytes, so
        // the interior loop can address them through one buffer resource
        const double span = ((double)p->rs + 2.0 * d.hr + 2.0) * std::max((double)m->ld * (double)es, (double)m->ld_mask);
        d.vec_ok = (m_vec ? 2 : 0) | (span < 2147483647.0 ? 4 : 0);
    }
    return d;
}

// ---------------------------------------------------------------------------
// Workspace layouts
// ---------------------------------------------------------------------------
// PLAIN form: integral-image units of kPlainChunk rows x kPlainW columns;
// stencil units of kPlainBand rows of one strip of 64*st_k columns.
constexpr int kPlainChunk = 128;
constexpr int kPlainBand = 16;

// Rows per unit of the PLAIN form's kernels (CFAR2D_PLAIN_CHUNK and
// CFAR2D_PLAIN_BAND override the defaults, for tuning).
static int plain_chunk()
{
    static const int v = env_int("CFAR2D_PLAIN_CHUNK", kPlainChunk);
    return v;
}
static int plain_band()
{
    static const int v = env_int("CFAR2D_PLAIN_BAND", kPlainBand);
    return v;
}
static int plain_xcd()
{
    static const int v = env_int("CFAR2D_PLAIN_XCD", 2) - 1;  // 1 (default): XCD-grouped stencil units
    return v;
}

static void plain_geometry(const cfar_map *m, PlainDesc &d)
{
    std::memset(&d, 0, sizeof d);
    const int64_t R = m->rows, F = m->cols;
    d.chunk = (int32_t)std::min<int64_t>(plain_chunk(), R);
    d.n_chunks = (int32_t)((R + d.chunk - 1) / d.chunk);
    d.n_strips = (int32_t)((F + kPlainW - 1) / kPlainW);
    const int hf = m->win.guard_f + m->win.train_f;
    // k = 4 while the halo costs less than half the strip, k = 8 up to the
    // widest window a 512-column strip holds, else the per-cell stencil
    d.st_k = hf <= 60 ? 4 : hf <= kMaxTiledHf ? 8 : 0;
    if (d.st_k) {
        const int a = std::max(4, (int)d.st_k);
        d.st_halo = (hf + 1 + a - 1) / a * a;
        d.st_tw = 64 * d.st_k - 2 * d.st_halo;
        d.st_strips = (int32_t)((F + d.st_tw - 1) / d.st_tw);
        // the interior rows run in chains of step hr - gr (two image rows per row
        // after a chain's first): bands of two chain steps (measured on the
        // 8192^2 map, hr - gr = 16: bands of 24-32 rows 0.65 ms, 16 rows 0.70,
        // 48 rows 0.68, 64 rows 0.70 ms)
        const int hr = m->win.guard_r + m->win.train_r, gr = m->win.guard_r;
        const int band = std::getenv("CFAR2D_PLAIN_BAND") ? plain_band()
                                                          : std::min(std::max(kPlainBand, 2 * (hr - gr)), 128);
        d.st_band = (int32_t)std::min<int64_t>(band, R);
        d.st_bands = (int32_t)((R + d.st_band - 1) / d.st_band);
        // maps of 8 strips or more: unit u of a band goes to strip group
        // u mod 8, so that the waves of one XCD (workgroups are dealt to the
        // XCDs in turn) keep to one group of columns and share its rows in L2
        if (plain_xcd() && d.st_strips >= 8) d.st_xcd = (d.st_strips + 7) / 8;
    }
}

static uint64_t plain_sat_units(const PlainDesc &d) { return (uint64_t)d.n_chunks * (uint64_t)d.n_strips; }
static uint64_t plain_st_units(const PlainDesc &d)
{
    if (!d.st_k) return 0;
    // a multiple of 8, so that every map's units start on the same XCD
    const uint64_t n = (uint64_t)d.st_bands * (uint64_t)(d.st_xcd ? 8 * d.st_xcd : d.st_strips);
    return (n + 7) / 8 * 8;
}
static uint64_t plain_carry_blocks(const cfar_map *m) { return (uint64_t)((m->cols + 255) / 256 + (m->rows + 255) / 256); }

// Device memory of the PLAIN form: a head (descriptors and unit tables,
// copied from the host; none for one map), then per map the integral image,
// the row carries, the column carries and the threshold table.
struct PlainLayout {
    size_t head_bytes = 0, off_desc = 0, off_sat = 0, off_st = 0, off_blk = 0;
    std::vector<size_t> s_off, left_off, v_off, lut_off;
    size_t total = 0;
};

static PlainLayout plain_layout(const cfar_map *maps, int n, std::vector<PlainDesc> &pd)
{
    PlainLayout L;
    pd.resize(n);
    if (n > 1) {
        L.off_desc = 0;
        L.off_sat = (size_t)n * sizeof(PlainDesc);
        L.off_st = L.off_sat + align_up((size_t)(n + 1) * 4, 16);
        L.off_blk = L.off_st + align_up((size_t)(n + 1) * 4, 16);
        L.head_bytes = align_up(L.off_blk + (size_t)(n + 1) * 4, 256);
    }
    size_t off = L.head_bytes;
    L.s_off.resize(n);
    L.left_off.resize(n);
    L.v_off.resize(n);
    L.lut_off.resize(n);
    for (int i = 0; i < n; ++i) {
        plain_geometry(&maps[i], pd[i]);
        L.s_off[i] = off;
        off += align_up((size_t)maps[i].rows * (size_t)maps[i].cols * 8, 256);
        L.left_off[i] = off;
        off += align_up((size_t)pd[i].n_strips * (size_t)maps[i].rows * 8, 256);
        L.v_off[i] = off;
        off += align_up((size_t)pd[i].n_chunks * (size_t)maps[i].cols * 8, 256);
        L.lut_off[i] = off;
        off += lut_bytes(&maps[i]);
    }
    L.total = off;
    return L;
}

static size_t plain_ws_bytes(const cfar_map *maps, int n)
{
    std::vector<PlainDesc> pd;
    return plain_layout(maps, n, pd).total;
}

struct TiledLayout {
    size_t head_bytes;     // header + descriptors + unit tables (copied from the host)
    size_t off_desc, off_base, off_umap, off_lut;
    std::vector<size_t> lut_off;  // per map, relative to ws
    size_t total;
};

static TiledLayout tiled_layout(const cfar_map *maps, int n, uint64_t total_units)
{
    TiledLayout L;
    L.off_desc = sizeof(BatchHeader);
    L.off_base = L.off_desc + (size_t)n * sizeof(MapDesc);
    L.off_umap = align_up(L.off_base + (size_t)n * 4, 16);
    L.head_bytes = align_up(L.off_umap + (size_t)total_units * 4, 256);
    L.off_lut = L.head_bytes;
    size_t off = L.off_lut;
    L.lut_off.resize(n);
    for (int i = 0; i < n; ++i) {
        L.lut_off[i] = off;
        off += lut_bytes(&maps[i]);
    }
    L.total = off;
    return L;
}

// LDS bytes per wave for the TILED kernel's row ring (CFAR2D_RING_BYTES
// overrides the default, for tuning).
static int ring_budget()
{
    static int v = -1;
    if (v < 0) {
        const char *e = std::getenv("CFAR2D_RING_BYTES");
        v = e ? std::max(0, std::atoi(e)) : kDefaultRingBytes;
    }
    return v;
}

// Work units below which the cost model shortens a map's units
// (CFAR2D_MIN_UNITS overrides the default, for tuning).
static int min_units()
{
    static int v = -1;
    if (v < 0) {
        const char *e = std::getenv("CFAR2D_MIN_UNITS");
        v = e ? std::max(0, std::atoi(e)) : kDefaultMinUnits;
    }
    return v;
}

// Maps of one kernel class (columns per lane k, dtype) and their work units.
struct KClass {
    int kset, dtype;  // kset 24: maps planned with k = 2 or 4; 8: k = 8
    bool out;         // maps of the class may write the optional outputs
    bool wide;        // maps whose guard ring exceeds the plan's budget (a launch of their own)
    uint32_t unit_off, units, blocks;
    int ring_bytes;   // LDS ring per wave of its launch (largest need among the maps)
};
static int class_slot(int kset, int dtype, bool out, bool wide)
{
    return (((wide ? 1 : 0) * 2 + (kset == 8 ? 1 : 0)) * 2 + dtype) * 2 + (out ? 1 : 0);
}
static bool has_outputs(const cfar_map *m) { return m->train_sum != nullptr || m->threshold != nullptr; }


// LDS one workgroup may use on the current device (queried once).
static int max_lds_per_block()
{
    static int v = 0;
    if (v == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        v = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
             prop.sharedMemPerBlock > 0)
                ? (int)prop.sharedMemPerBlock
                : 65536;
    }
    return v;
}

// LDS ring bytes map m needs under its plan's budget (and what one
// workgroup can hold besides the prefix rows).
// The guard ring of a map, within the plan's budget; a ring the budget does
// not hold but kRingStretchBytes does is given its own size all the same
// (unless the plan turns the ring off with a budget of 0): the loop without
// it loads five rows per row step, which costs more than the waves the larger
// LDS share takes (guard 8 on a 16384^2 FP32 map: 0.98 ms without the ring,
// 0.63 ms with an 18 KiB one).
static int map_ring_bytes(const cfar_map *m, const Plan &p)
{
    const int hr = m->win.guard_r + m->win.train_r;
    const int room = std::max(max_lds_per_block() - (int)fused_lds_bytes(kset_of(p.k), 0), 0);
    const int need = ring_bytes_needed(p.k, m->dtype, hr, m->win.guard_r, std::min(p.ring_bytes, room));
    if (need > 0 || p.ring_bytes <= 0) return need;
    return ring_bytes_needed(p.k, m->dtype, hr, m->win.guard_r, std::min(std::max(p.ring_bytes, kRingStretchBytes), room));
}

// ---------------------------------------------------------------------------
// Batch contexts: pinned staging buffers (double-buffered per stream and
// workspace) and the hipGraphs captured on them.
// ---------------------------------------------------------------------------
struct Slot {
    void *pinned = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool recorded = false;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    // signature of the captured graph
    size_t sig_head = 0;
    uint64_t sig_layout = 0;
    uint32_t sig_units = 0, sig_n = 0;
    ~Slot()
    {
        if (recorded && done) (void)hipEventSynchronize(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (done) (void)hipEventDestroy(done);
        if (pinned) (void)hipHostFree(pinned);
    }
};
// Kernel classes after the first run on side streams forked from (and
// joined back into) the caller's stream, so a small class fills the tail of
// a large one.
constexpr int kSideStreams = 5;
struct BatchCtx {
    Slot slot[2];
    int next = 0;
    std::mutex mu;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr, join[kSideStreams] = {};
    ~BatchCtx()
    {
        for (int i = 0; i < kSideStreams; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join[i]) (void)hipEventDestroy(join[i]);
        }
        if (fork) (void)hipEventDestroy(fork);
    }
    int ensure_side(int n)
    {
        if (!fork) {
            hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
            if (e != hipSuccess) return hip_error(e, "hipEventCreate(fork)");
        }
        for (int i = 0; i < n && i < kSideStreams; ++i) {
            if (!side[i]) {
                hipError_t e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
                if (e != hipSuccess) return hip_error(e, "hipStreamCreate(side)");
            }
            if (!join[i]) {
                hipError_t e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
                if (e != hipSuccess) return hip_error(e, "hipEventCreate(join)");
            }
        }
        return CFAR_OK;
    }
};
static std::mutex g_ctx_mu;
// Never destroyed: contexts hold HIP objects, which must not be released
// from static destructors after the runtime has gone at process exit.
static auto &g_ctx = *new std::map<std::pair<void *, void *>, std::unique_ptr<BatchCtx>>();

// Forget the batch context of (stream, ws): its staging buffers, graphs and
// side streams are freed once its last batch has finished.
void drop_batch_ctx(hipStream_t s, void *ws)
{
    std::unique_ptr<BatchCtx> p;
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        auto it = g_ctx.find(std::make_pair((void *)s, ws));
        if (it == g_ctx.end()) return;
        p = std::move(it->second);
        g_ctx.erase(it);
    }
    std::lock_guard<std::mutex> lk(p->mu);
}

static BatchCtx *get_ctx(hipStream_t s, void *ws)
{
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto &p = g_ctx[std::make_pair((void *)s, ws)];
    if (!p) p.reset(new BatchCtx());
    return p.get();
}

static int slot_reserve(Slot &sl, size_t bytes)
{
    if (sl.recorded) {
        hipError_t e = hipEventSynchronize(sl.done);
        if (e != hipSuccess) return hip_error(e, "hipEventSynchronize(staging)");
        sl.recorded = false;
    }
    if (!sl.done) {
        hipError_t e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_error(e, "hipEventCreate");
    }
    if (sl.cap < bytes) {
        if (sl.exec) { (void)hipGraphExecDestroy(sl.exec); sl.exec = nullptr; }
        if (sl.graph) { (void)hipGraphDestroy(sl.graph); sl.graph = nullptr; }
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pinned = nullptr;
        size_t cap = std::max<size_t>(bytes, 64 << 10);
        hipError_t e = hipHostMalloc(&sl.pinned, cap, hipHostMallocDefault);
        if (e != hipSuccess) { sl.cap = 0; return hip_error(e, "hipHostMalloc(staging)"); }
        sl.cap = cap;
    }
    return CFAR_OK;
}

// Enqueue: descriptor copy, table kernel, one persistent kernel per class.
static int enqueue_tiled_batch(BatchCtx *ctx, const Slot &sl, const TiledLayout &L, char *ws, uint32_t n,
                               const std::vector<KClass> &classes, hipStream_t stream)
{
    hipError_t e = hipMemcpyAsync(ws, sl.pinned, L.head_bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(descriptors)");
    MapDesc dummy;
    std::memset(&dummy, 0, sizeof dummy);
    const MapDesc *descs = (const MapDesc *)(ws + L.off_desc);
    BatchHeader *hdr = (BatchHeader *)ws;
    e = launch_lut(descs, sizeof(MapDesc), dummy, (int)n, hdr->counter, stream);
    if (e != hipSuccess) return hip_error(e, "launch(lut_kernel)");
    e = timing_mark(g_timing.start, stream);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    // classes 1.. on side streams (a stream with the default handle has no
    // side streams: it serialises with every other stream anyway)
    const int n_side = stream ? std::min<int>((int)classes.size() - 1, kSideStreams) : 0;
    if (n_side > 0) {
        int rc = ctx->ensure_side(n_side);
        if (rc != CFAR_OK) return rc;
        e = hipEventRecord(ctx->fork, stream);
        if (e != hipSuccess) return hip_error(e, "hipEventRecord(fork)");
        for (int i = 0; i < n_side; ++i) {
            e = hipStreamWaitEvent(ctx->side[i], ctx->fork, 0);
            if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent(fork)");
        }
    }
    for (size_t ci = 0; ci < classes.size(); ++ci) {
        const KClass &c = classes[ci];
        const int si = (int)ci - 1;
        hipStream_t cs = (si >= 0 && si < n_side) ? ctx->side[si] : stream;
        FusedArgs a;
        std::memset(&a, 0, sizeof a);
        a.descs = descs;
        a.unit_base = (const uint32_t *)(ws + L.off_base);
        a.unit_map = (const uint32_t *)(ws + L.off_umap) + c.unit_off;
        a.counter = &hdr->counter[class_slot(c.kset, c.dtype, c.out, c.wide)];
        a.total_units = c.units;
        a.n_maps = n;
        a.ring_bytes = c.ring_bytes;
        e = launch_fused(a, c.kset, c.dtype, c.out, cs);
        if (e != hipSuccess) return hip_error(e, "launch(fused_kernel)");
    }
    for (int i = 0; i < n_side; ++i) {
        e = hipEventRecord(ctx->join[i], ctx->side[i]);
        if (e != hipSuccess) return hip_error(e, "hipEventRecord(join)");
        e = hipStreamWaitEvent(stream, ctx->join[i], 0);
        if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent(join)");
    }
    e = timing_mark(g_timing.stop, stream);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    if (g_timing.on) g_timing.recorded = true;
    return CFAR_OK;
}

static int run_tiled_batch(const cfar_map *maps, int n, int flags, void *ws, size_t ws_bytes, hipStream_t stream,
                           const cfar_plan *forced)
{
    std::vector<Plan> plans(n);
    uint64_t total_units = 0;
    // A batch whose maps already give the chip kBatchFullUnits work units
    // keeps every map's units at full length: shortening a small map's units
    // (which spreads it over more waves when it runs alone) only adds warm-up
    // rows here.  Otherwise the maps are planned as they would be alone.
    bool spread = n == 1 || forced;
    for (;;) {
        total_units = 0;
        for (int i = 0; i < n; ++i) {
            cfar_plan cp = forced ? *forced : choose_plan(&maps[i], spread);
            if (!plan_geometry(&maps[i], cp.k_cols, cp.rows_per_unit, &plans[i], cp.ring_bytes))
                return set_error(CFAR_EINVAL, "map %d: no valid tile plan", i);
            total_units += units_of(plans[i]);
        }
        if (spread || total_units >= (uint64_t)kBatchFullUnits) break;
        spread = true;
    }
    if (total_units >= (uint64_t)1 << 31) return set_error(CFAR_EINVAL, "batch has too many work units");
    TiledLayout L = tiled_layout(maps, n, total_units);
    if (ws_bytes < L.total)
        return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, L.total);
    if (!ws) return set_error(CFAR_EINVAL, "ws is NULL");

    // Kernel classes (k, dtype), each with its own persistent launch; inside a
    // class larger maps come first (better tail balance).  A map's result does
    // not depend on the order or on the other maps.
    std::vector<KClass> classes;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < n; ++i) {
        const int ks = kset_of(plans[i].k), dt = maps[i].dtype;
        const bool out = has_outputs(&maps[i]);
        const bool wide = map_ring_bytes(&maps[i], plans[i]) > plans[i].ring_bytes;
        size_t c = 0;
        while (c < classes.size() && !(classes[c].kset == ks && classes[c].dtype == dt && classes[c].out == out &&
                                       classes[c].wide == wide))
            ++c;
        if (c == classes.size()) {
            KClass kc;
            kc.kset = ks; kc.dtype = dt; kc.out = out; kc.wide = wide; kc.unit_off = 0; kc.units = 0; kc.blocks = 0;
            kc.ring_bytes = 0;
            classes.push_back(kc);
            members.emplace_back();
        }
        members[c].push_back(i);
        classes[c].units += (uint32_t)units_of(plans[i]);
        classes[c].ring_bytes = std::max(classes[c].ring_bytes, map_ring_bytes(&maps[i], plans[i]));
    }
    {
        std::vector<size_t> corder(classes.size());
        std::iota(corder.begin(), corder.end(), 0);
        std::stable_sort(corder.begin(), corder.end(),
                         [&](size_t a, size_t b) { return classes[a].units > classes[b].units; });
        std::vector<KClass> c2;
        std::vector<std::vector<int>> m2;
        for (size_t c : corder) { c2.push_back(classes[c]); m2.push_back(members[c]); }
        classes.swap(c2);
        members.swap(m2);
    }
    uint32_t off = 0;
    for (size_t c = 0; c < classes.size(); ++c) {
        classes[c].unit_off = off;
        off += classes[c].units;
        const int resident =
            fused_resident_blocks(classes[c].kset, classes[c].dtype, classes[c].out, classes[c].ring_bytes);
        classes[c].blocks = (uint32_t)std::min<uint64_t>(classes[c].units, (uint64_t)resident);
        std::stable_sort(members[c].begin(), members[c].end(),
                         [&](int a, int b) { return units_of(plans[a]) > units_of(plans[b]); });
    }

    BatchCtx *ctx = get_ctx(stream, ws);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Slot &sl = ctx->slot[ctx->next];
    ctx->next ^= 1;
    int rc = slot_reserve(sl, L.head_bytes);
    if (rc != CFAR_OK) return rc;

    char *h = (char *)sl.pinned;
    std::memset(h, 0, sizeof(BatchHeader));
    BatchHeader *hdr = (BatchHeader *)h;
    hdr->n_maps = (uint32_t)n;
    hdr->total_units = (uint32_t)total_units;
    MapDesc *descs = (MapDesc *)(h + L.off_desc);
    uint32_t *ubase = (uint32_t *)(h + L.off_base);
    uint32_t *umap = (uint32_t *)(h + L.off_umap);
    for (int i = 0; i < n; ++i) descs[i] = make_desc(&maps[i], &plans[i], (double *)((char *)ws + L.lut_off[i]));
    for (size_t c = 0; c < classes.size(); ++c) {
        uint32_t u = 0;  // unit numbers are local to the class
        for (int i : members[c]) {
            ubase[i] = u;
            const uint64_t cnt = units_of(plans[i]);
            for (uint64_t k = 0; k < cnt; ++k) umap[classes[c].unit_off + u++] = (uint32_t)i;
        }
    }
    uint64_t sig = 1469598103934665603ull;  // FNV-1a over the class layout
    for (const KClass &c : classes) {
        const uint32_t f[7] = {(uint32_t)c.kset, (uint32_t)c.dtype, (uint32_t)c.out, c.unit_off, c.units, c.blocks,
                               (uint32_t)c.ring_bytes};
        for (uint32_t v : f) { sig ^= v; sig *= 1099511628211ull; }
    }

    const bool use_graph = (flags & CFAR_BATCH_GRAPH) && stream != nullptr && !g_timing.on;
    if (use_graph) {
        const bool match = sl.exec && sl.sig_head == L.head_bytes && sl.sig_units == total_units &&
                           sl.sig_layout == sig && sl.sig_n == (uint32_t)n;
        if (!match) {
            if (sl.exec) { (void)hipGraphExecDestroy(sl.exec); sl.exec = nullptr; }
            if (sl.graph) { (void)hipGraphDestroy(sl.graph); sl.graph = nullptr; }
            hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
            rc = enqueue_tiled_batch(ctx, sl, L, (char *)ws, (uint32_t)n, classes, stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(stream, &g);
            if (rc != CFAR_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
            if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) { (void)hipGraphDestroy(g); sl.exec = nullptr; return hip_error(e, "hipGraphInstantiate"); }
            sl.graph = g;
            sl.sig_head = L.head_bytes;
            sl.sig_units = (uint32_t)total_units;
            sl.sig_layout = sig;
            sl.sig_n = (uint32_t)n;
        }
        hipError_t e = hipGraphLaunch(sl.exec, stream);
        if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    } else {
        rc = enqueue_tiled_batch(ctx, sl, L, (char *)ws, (uint32_t)n, classes, stream);
        if (rc != CFAR_OK) return rc;
    }
    hipError_t e = hipEventRecord(sl.done, stream);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord");
    sl.recorded = true;
    return CFAR_OK;
}

// Single map, TILED: descriptor travels as a kernel argument; ws holds the
// work counter and the threshold table.
static int run_tiled_single(const cfar_map *m, const cfar_plan &cp, void *ws, size_t ws_bytes, hipStream_t stream)
{
    Plan p;
    if (!plan_geometry(m, cp.k_cols, cp.rows_per_unit, &p, cp.ring_bytes))
        return set_error(CFAR_EINVAL, "no valid tile plan");
    const size_t need = sizeof(BatchHeader) + lut_bytes(m);
    if (ws_bytes < need) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, need);
    if (!ws) return set_error(CFAR_EINVAL, "ws is NULL");
    const uint64_t units = units_of(p);
    if (units >= (uint64_t)1 << 31) return set_error(CFAR_EINVAL, "map has too many work units");
    BatchHeader *hdr = (BatchHeader *)ws;
    uint32_t *counter = hdr->counter;
    double *lut = (double *)((char *)ws + sizeof(BatchHeader));
    FusedArgs a;
    std::memset(&a, 0, sizeof a);
    a.single = make_desc(m, &p, lut);
    a.counter = counter;
    a.total_units = (uint32_t)units;
    a.n_maps = 1;
    a.ring_bytes = map_ring_bytes(m, p);
    hipError_t e = launch_lut(nullptr, 0, a.single, 1, counter, stream);
    if (e != hipSuccess) return hip_error(e, "launch(lut_kernel)");
    e = timing_mark(g_timing.start, stream);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    e = launch_fused(a, kset_of(p.k), m->dtype, has_outputs(m), stream);
    if (e != hipSuccess) return hip_error(e, "launch(fused_kernel)");
    e = timing_mark(g_timing.stop, stream);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    if (g_timing.on) g_timing.recorded = true;
    return CFAR_OK;
}

// Single map, TILED, its plan chosen as cfar2d does (the allocation-free
// entry point runs it on its static workspace).
int tiled_single_ws(const cfar_map *m, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return run_tiled_single(m, choose_plan(m), ws, ws_bytes, stream);
}

size_t tiled_single_ws_bytes(const cfar_map *m) { return sizeof(BatchHeader) + lut_bytes(m); }

// Single map, DIRECT: table, then every cell sums its own window.  Kernel
// timing (if on) starts before the first map's stencil and stops after the
// last one's.
static int run_direct_single(const cfar_map *m, void *ws, size_t ws_bytes, hipStream_t stream, bool first = true,
                             bool last = true)
{
    const size_t need = lut_bytes(m);
    if (ws_bytes < need) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, need);
    if (!ws) return set_error(CFAR_EINVAL, "ws is NULL");
    MapDesc d = make_desc(m, nullptr, (double *)ws);
    hipError_t e = launch_lut(nullptr, 0, d, 1, nullptr, stream);
    if (e != hipSuccess) return hip_error(e, "launch(lut_kernel)");
    if (first && (e = timing_mark(g_timing.start, stream)) != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    e = launch_stencil_direct(d, stream);
    if (e != hipSuccess) return hip_error(e, "launch(stencil_direct)");
    if (last) {
        if ((e = timing_mark(g_timing.stop, stream)) != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
        if (g_timing.on) g_timing.recorded = true;
    }
    return CFAR_OK;
}

// PLAIN form over n maps: the head (for more than one map) through the
// pinned staging of the batch context, the threshold tables, then the
// integral image and the stencil, each one launch over every map's units.
// Maps too wide for the strip stencil take the per-cell stencil, one launch
// each.
static int run_plain_batch(const cfar_map *maps, int n, void *ws, size_t ws_bytes, hipStream_t stream)
{
    std::vector<PlainDesc> pd;
    const PlainLayout L = plain_layout(maps, n, pd);
    if (ws_bytes < L.total) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, L.total);
    if (!ws) return set_error(CFAR_EINVAL, "ws is NULL");
    char *w = (char *)ws;
    PlainArgs a;
    std::memset(&a, 0, sizeof a);
    uint64_t sat_units = 0, st_units = 0, blocks = 0;
    int k_mask = 0;
    bool any_out = false;
    std::vector<uint32_t> sat_base(n + 1), st_base(n + 1), blk_base(n + 1);
    for (int i = 0; i < n; ++i) {
        PlainDesc &d = pd[i];
        d.m = make_desc(&maps[i], nullptr, (double *)(w + L.lut_off[i]));
        d.S = (double *)(w + L.s_off[i]);
        d.left = (double *)(w + L.left_off[i]);
        d.V = (double *)(w + L.v_off[i]);
        sat_base[i] = (uint32_t)sat_units;
        st_base[i] = (uint32_t)st_units;
        blk_base[i] = (uint32_t)blocks;
        sat_units += plain_sat_units(d);
        st_units += plain_st_units(d);
        blocks += plain_carry_blocks(&maps[i]);
        k_mask |= d.st_k;
        any_out = any_out || (d.st_k && has_outputs(&maps[i]));
    }
    if (sat_units >= (uint64_t)1 << 31 || st_units >= (uint64_t)1 << 31 || blocks >= (uint64_t)1 << 31)
        return set_error(CFAR_EINVAL, "batch has too many work units");
    sat_base[n] = (uint32_t)sat_units;
    st_base[n] = (uint32_t)st_units;
    blk_base[n] = (uint32_t)blocks;
    a.n_maps = (uint32_t)n;
    a.sat_units = (uint32_t)sat_units;
    a.st_units = (uint32_t)st_units;
    a.carry_blocks = (uint32_t)blocks;
    hipError_t e;
    if (n == 1) {
        a.single = pd[0];
        e = launch_lut(nullptr, 0, pd[0].m, 1, nullptr, stream);
        if (e != hipSuccess) return hip_error(e, "launch(lut_kernel)");
    } else {
        BatchCtx *ctx = get_ctx(stream, ws);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Slot &sl = ctx->slot[ctx->next];
        ctx->next ^= 1;
        int rc = slot_reserve(sl, L.head_bytes);
        if (rc != CFAR_OK) return rc;
        char *h = (char *)sl.pinned;
        std::memcpy(h + L.off_desc, pd.data(), (size_t)n * sizeof(PlainDesc));
        std::memcpy(h + L.off_sat, sat_base.data(), (size_t)(n + 1) * 4);
        std::memcpy(h + L.off_st, st_base.data(), (size_t)(n + 1) * 4);
        std::memcpy(h + L.off_blk, blk_base.data(), (size_t)(n + 1) * 4);
        e = hipMemcpyAsync(ws, sl.pinned, L.head_bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(descriptors)");
        e = hipEventRecord(sl.done, stream);
        if (e != hipSuccess) return hip_error(e, "hipEventRecord");
        sl.recorded = true;
        a.descs = (const PlainDesc *)(w + L.off_desc);
        a.sat_base = (const uint32_t *)(w + L.off_sat);
        a.st_base = (const uint32_t *)(w + L.off_st);
        a.blk_base = (const uint32_t *)(w + L.off_blk);
        MapDesc dummy;
        std::memset(&dummy, 0, sizeof dummy);
        e = launch_lut(a.descs, sizeof(PlainDesc), dummy, n, nullptr, stream);
        if (e != hipSuccess) return hip_error(e, "launch(lut_kernel)");
    }
    if ((e = timing_mark(g_timing.start, stream)) != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    e = launch_plain(a, k_mask, true, any_out, stream);
    if (e != hipSuccess) return hip_error(e, "launch(plain)");
    for (int i = 0; i < n; ++i) {
        if (pd[i].st_k) continue;
        e = launch_stencil_plain(pd[i].m, pd[i].S, stream);
        if (e != hipSuccess) return hip_error(e, "launch(stencil_plain)");
    }
    if ((e = timing_mark(g_timing.stop, stream)) != hipSuccess) return hip_error(e, "hipEventRecord(timing)");
    if (g_timing.on) g_timing.recorded = true;
    return CFAR_OK;
}

// sat2d, PLAIN form: the integral-image kernels of the PLAIN form on one map
// (no stencil); ws holds the row and column carries.
static size_t plain_sat_ws_bytes(int64_t rows, int64_t cols)
{
    const int64_t chunk = std::min<int64_t>(plain_chunk(), rows);
    const int64_t nc = (rows + chunk - 1) / chunk, ns = (cols + kPlainW - 1) / kPlainW;
    return align_up((size_t)(ns * rows) * 8, 256) + align_up((size_t)(nc * cols) * 8, 256);
}

static int run_plain_sat2d(const void *x, int dtype, int64_t rows, int64_t cols, int64_t ld, double *sat, void *ws,
                           hipStream_t stream)
{
    PlainArgs a;
    std::memset(&a, 0, sizeof a);
    PlainDesc &d = a.single;
    cfar_map m;
    std::memset(&m, 0, sizeof m);
    m.x = x;
    m.dtype = dtype;
    m.rows = rows;
    m.cols = cols;
    m.ld = ld;
    m.win.pfa = 0.5;
    plain_geometry(&m, d);
    d.m.x = x;
    d.m.dtype = dtype;
    d.m.rows = (int32_t)rows;
    d.m.cols = (int32_t)cols;
    d.m.ld = ld;
    d.S = sat;
    d.left = (double *)ws;
    d.V = (double *)((char *)ws + align_up((size_t)(d.n_strips * rows) * 8, 256));
    a.n_maps = 1;
    a.sat_units = (uint32_t)plain_sat_units(d);
    a.carry_blocks = (uint32_t)plain_carry_blocks(&m);
    const hipError_t e = launch_plain(a, 0, false, false, stream);
    return e == hipSuccess ? CFAR_OK : hip_error(e, "launch(plain sat2d)");
}

// ---------------------------------------------------------------------------
// SAT workspace
// ---------------------------------------------------------------------------
size_t sat_ws_bytes(int64_t rows, int64_t cols)
{
    const int64_t nI = (rows + kSatTH - 1) / kSatTH, nJ = (cols + kSatTW - 1) / kSatTW;
    const size_t t = (size_t)(nI * nJ);
    return align_up(t * kSatTH * 8, 256) * 2 + align_up(t * kSatTW * 8, 256) * 2 + align_up(t * 8, 256) * 2;
}

SatWs sat_ws_layout(void *ws, int64_t rows, int64_t cols)
{
    SatWs s;
    s.nI = (rows + kSatTH - 1) / kSatTH;
    s.nJ = (cols + kSatTW - 1) / kSatTW;
    const size_t t = (size_t)(s.nI * s.nJ);
    char *p = (char *)ws;
    s.agg_row = (double *)p; p += align_up(t * kSatTH * 8, 256);
    s.left = (double *)p; p += align_up(t * kSatTH * 8, 256);
    s.agg_cs = (double *)p; p += align_up(t * kSatTW * 8, 256);
    s.top = (double *)p; p += align_up(t * kSatTW * 8, 256);
    s.agg_tot = (double *)p; p += align_up(t * 8, 256);
    s.rt = (double *)p;
    return s;
}

}  // namespace cfar

using namespace cfar;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *cfar_last_error(void) { return g_err.c_str(); }

const char *cfar_version(void) { return "cfar2d-mi355x 0.1 (gfx950)"; }

size_t sat2d_bytes(int64_t rows, int64_t cols, int32_t form)
{
    if (rows < 1 || cols < 1 || rows > kMaxDim || cols > kMaxDim) return 0;
    if (form == CFAR_FORM_PLAIN) return (size_t)rows * (size_t)cols * 8;
    if (form == CFAR_FORM_TILED) {
        const int64_t nI32 = (rows + kLine - 1) / kLine, nJ32 = (cols + kLine - 1) / kLine;
        return align_up((size_t)rows * cols * 4, 256) + align_up((size_t)nI32 * cols * 8, 256) +
               align_up((size_t)nJ32 * rows * 8, 256);
    }
    return 0;
}

size_t sat2d_workspace_bytes(int64_t rows, int64_t cols, int32_t form)
{
    if (rows < 1 || cols < 1 || rows > kMaxDim || cols > kMaxDim) return 0;
    if (form == CFAR_FORM_PLAIN) return plain_sat_ws_bytes(rows, cols);
    if (form != CFAR_FORM_TILED) return 0;
    return sat_ws_bytes(rows, cols);
}

int sat2d(const void *x, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, int32_t form, void *sat_out,
          size_t sat_bytes, void *ws, size_t ws_bytes, void *stream)
{
    if (dtype != CFAR_F32 && dtype != CFAR_F64) return set_error(CFAR_EINVAL, "unknown dtype %d", dtype);
    if (form != CFAR_FORM_PLAIN && form != CFAR_FORM_TILED) return set_error(CFAR_EINVAL, "unknown form %d", form);
    if (rows < 1 || cols < 1 || rows > kMaxDim || cols > kMaxDim)
        return set_error(CFAR_EINVAL, "rows and cols must lie in [1, 2^30]");
    if (ld < cols) return set_error(CFAR_EINVAL, "ld < cols");
    if (!x || !sat_out || !ws) return set_error(CFAR_EINVAL, "NULL pointer argument");
    const size_t need = sat2d_bytes(rows, cols, form);
    if (sat_bytes < need) return set_error(CFAR_ENOSPC, "sat_bytes %zu < %zu needed", sat_bytes, need);
    const size_t wneed = form == CFAR_FORM_PLAIN ? plain_sat_ws_bytes(rows, cols) : sat_ws_bytes(rows, cols);
    if (ws_bytes < wneed) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, wneed);
    if (form == CFAR_FORM_PLAIN) {
        if (rows * ((cols + kPlainW - 1) / kPlainW) >= ((int64_t)1 << 31) ||
            ((rows + plain_chunk() - 1) / plain_chunk()) * ((cols + kPlainW - 1) / kPlainW) >= ((int64_t)1 << 31))
            return set_error(CFAR_EINVAL, "map too large for sat2d");
        return run_plain_sat2d(x, dtype, rows, cols, ld, (double *)sat_out, ws, (hipStream_t)stream);
    }
    SatWs sw = sat_ws_layout(ws, rows, cols);
    hipError_t e = launch_sat2d(x, dtype, rows, cols, ld, form, sat_out, sw, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "launch(sat2d)");
    return CFAR_OK;
}

size_t cfar_workspace_bytes(const cfar_map *maps, int32_t n, int32_t form)
{
    if (!maps || n < 1) { set_error(CFAR_EINVAL, "maps is NULL or n < 1"); return 0; }
    for (int i = 0; i < n; ++i)
        if (validate_map(&maps[i], i, form) != CFAR_OK) return 0;
    if (form == CFAR_FORM_PLAIN) return plain_ws_bytes(maps, n);
    if (form == CFAR_FORM_DIRECT) {
        size_t need = 0;
        for (int i = 0; i < n; ++i) need = std::max(need, lut_bytes(&maps[i]));
        return need;
    }
    uint64_t total_units = 0;
    for (int i = 0; i < n; ++i) {
        cfar_plan cp = choose_plan(&maps[i]);
        Plan p;
        if (!plan_geometry(&maps[i], cp.k_cols, cp.rows_per_unit, &p)) return 0;
        total_units += units_of(p);
    }
    // enough for the batch layout; a single map needs less
    return tiled_layout(maps, n, total_units).total;
}

int cfar2d(const cfar_map *m, int32_t form, void *ws, size_t ws_bytes, void *stream)
{
    int rc = validate_map(m, 0, form);
    if (rc != CFAR_OK) return rc;
    if (form == CFAR_FORM_PLAIN) return run_plain_batch(m, 1, ws, ws_bytes, (hipStream_t)stream);
    if (form == CFAR_FORM_DIRECT) return run_direct_single(m, ws, ws_bytes, (hipStream_t)stream);
    return run_tiled_single(m, choose_plan(m), ws, ws_bytes, (hipStream_t)stream);
}

int cfar2d_with_plan(const cfar_map *m, const cfar_plan *plan, void *ws, size_t ws_bytes, void *stream)
{
    int rc = validate_map(m, 0, CFAR_FORM_TILED);
    if (rc != CFAR_OK) return rc;
    if (!plan || !plan_valid(m, plan)) return set_error(CFAR_EINVAL, "invalid plan for this map");
    return run_tiled_single(m, *plan, ws, ws_bytes, (hipStream_t)stream);
}

int cfar2d_batched(const cfar_map *maps, int32_t n, int32_t form, int32_t flags, void *ws, size_t ws_bytes,
                   void *stream)
{
    if (!maps || n < 1) return set_error(CFAR_EINVAL, "maps is NULL or n < 1");
    if (flags & ~CFAR_BATCH_GRAPH) return set_error(CFAR_EINVAL, "unknown flags 0x%x", flags);
    for (int i = 0; i < n; ++i) {
        int rc = validate_map(&maps[i], i, form);
        if (rc != CFAR_OK) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    if (form == CFAR_FORM_PLAIN) return run_plain_batch(maps, n, ws, ws_bytes, s);
    if (form == CFAR_FORM_DIRECT) {  // one table + one stencil launch per map, in order on the stream
        size_t need = 0;
        for (int i = 0; i < n; ++i) need = std::max(need, lut_bytes(&maps[i]));
        if (ws_bytes < need) return set_error(CFAR_ENOSPC, "ws_bytes %zu < %zu needed", ws_bytes, need);
        for (int i = 0; i < n; ++i) {
            int rc = run_direct_single(&maps[i], ws, ws_bytes, s, i == 0, i == n - 1);
            if (rc != CFAR_OK) return rc;
        }
        return CFAR_OK;
    }
    return run_tiled_batch(maps, n, flags, ws, ws_bytes, s, nullptr);
}

int cfar_plan_for(const cfar_map *m, cfar_plan *out)
{
    int rc = validate_map(m, 0, CFAR_FORM_TILED);
    if (rc != CFAR_OK) return rc;
    if (!out) return set_error(CFAR_EINVAL, "out is NULL");
    *out = choose_plan(m);
    return CFAR_OK;
}

// Plan table: one rule per line,
//   dtype cols_lo cols_hi rows_lo rows_hi hf_lo hf_hi hr_lo hr_hi k rows_per_unit [ring_bytes]
// dtype = f32 | f64 | any; '#' starts a comment.  First matching rule wins.
int cfar_plan_load(const char *path)
{
    std::vector<PlanRule> rules;
    if (path && *path) {
        std::ifstream f(path);
        if (!f) return set_error(CFAR_EINVAL, "cannot open plan table %s", path);
        std::string line;
        int ln = 0;
        while (std::getline(f, line)) {
            ++ln;
            const size_t hash = line.find('#');
            if (hash != std::string::npos) line.resize(hash);
            std::istringstream is(line);
            std::string dt;
            if (!(is >> dt)) continue;
            PlanRule r;
            long long c0, c1, r0, r1;
            if (!(is >> c0 >> c1 >> r0 >> r1 >> r.hf_lo >> r.hf_hi >> r.hr_lo >> r.hr_hi >> r.k >> r.rs))
                return set_error(CFAR_EINVAL, "%s:%d: malformed rule", path, ln);
            if (!(is >> r.ring_bytes)) r.ring_bytes = -1;
            if (r.ring_bytes < -1 || r.ring_bytes > 65536)
                return set_error(CFAR_EINVAL, "%s:%d: ring_bytes must be -1 or in [0, 65536]", path, ln);
            r.c_lo = c0; r.c_hi = c1; r.r_lo = r0; r.r_hi = r1;
            if (dt == "f32") r.dtype = 0;
            else if (dt == "f64") r.dtype = 1;
            else if (dt == "any") r.dtype = -1;
            else return set_error(CFAR_EINVAL, "%s:%d: dtype must be f32, f64 or any", path, ln);
            if (!(r.k == 2 || r.k == 4 || r.k == 8) || r.rs < 1 || r.rs > 4096)
                return set_error(CFAR_EINVAL, "%s:%d: k must be 2, 4 or 8 and rows_per_unit in [1, 4096]", path, ln);
            rules.push_back(r);
        }
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_rules.swap(rules);
    return CFAR_OK;
}

int cfar_timing_enable(int32_t on)
{
    if (on && !g_timing.start) {
        hipError_t e = hipEventCreate(&g_timing.start);
        if (e != hipSuccess) return hip_error(e, "hipEventCreate");
        e = hipEventCreate(&g_timing.stop);
        if (e != hipSuccess) return hip_error(e, "hipEventCreate");
    }
    g_timing.on = on != 0;
    g_timing.recorded = false;
    return CFAR_OK;
}

int cfar_timing_read(double *kernel_ms)
{
    if (!kernel_ms) return set_error(CFAR_EINVAL, "kernel_ms is NULL");
    if (!g_timing.recorded) return set_error(CFAR_EINVAL, "no timed launch on this thread");
    hipError_t e = hipEventSynchronize(g_timing.stop);
    if (e != hipSuccess) return hip_error(e, "hipEventSynchronize(timing)");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, g_timing.start, g_timing.stop);
    if (e != hipSuccess) return hip_error(e, "hipEventElapsedTime");
    *kernel_ms = ms;
    return CFAR_OK;
}

}  // extern "C"
