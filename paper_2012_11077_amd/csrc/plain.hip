// PLAIN CA-CFAR for gfx950: the paper's route (Sec. II.B).  The integral
// image of eq. (3) is written to device memory in FP64; the four corners of
// eq. (4) for the outer and the guard window of every cell are read back from
// it, then the threshold of eq. (2) and the decision of eq. (1).
//
// Integral image.  A map is cut into work units of `chunk` rows by kPlainW =
// 256 columns (chunk c, strip s; lane l holds columns 256 s + 4 l .. + 3).
// For a cell (i, j) of unit (c, s) with first row r0 and first column j0:
//
//   S(i,j) = A(c,s) + L(s,i) + V(c,j) + P(i,j)
//
//   P(i,j) = X summed over rows r0..i,   columns j0..j   (the unit's cells)
//   V(c,j) = X summed over rows 0..r0-1, columns j0..j
//   L(s,i) = X summed over rows r0..i,   columns 0..j0-1
//   A(c,s) = X summed over rows 0..r0-1, columns 0..j0-1
//
// plain_aggregate (per unit) writes the total of every row over the unit's
// columns (left[s][i]) and the strip prefix of the unit's column totals
// (V[c][j], the last row of P).  plain_carry turns both into exclusive sums:
// left[s][i] = X summed over row i, columns 0..j0-1 (a scan over the
// strips), V[c][j] = the V(c,j) above (a scan over the chunks).
// plain_finalize (per unit) builds P row by row (in-lane prefix, then a wave
// scan, added to running column sums), L as a running sum of left, A as the
// sum of V at the last columns of the strips to the left, and writes S.
// No unit waits for another: the three kernels are ordered by the stream.
//
// Stencil.  plain_stencil: per work unit (a band of rows of one strip of
// 64*K columns with a halo of H >= hf + 1 columns on each side), for every
// row: the four integral-image rows of eq. (4)'s row corners (the clipped
// rows; row -1 reads zero), their difference per column (the window's rows
// summed over columns 0..j), published to LDS, and the column corners read
// back at +h and -h-1 (clipped: a position left of the map reads zero, one
// right of it the value at the map's last column).  Units are handed out in
// order band by band and every wave strides through them, so the integral
// image rows a band needs are read while the neighbouring bands' waves still
// hold them in L2.
#include "internal.h"
#include "devutil.h"

#include <algorithm>
#include <cmath>

// Rows of integral-image loads in flight per wave in the stencil.
#ifndef CFAR_PLAIN_PD
#define CFAR_PLAIN_PD 2
#endif
// Interior rows of the stencil in chains of step hr - gr (two image rows
// loaded per row instead of four).
#ifndef CFAR_PLAIN_CHAIN
#define CFAR_PLAIN_CHAIN 1
#endif

namespace cfar {

namespace {

using namespace dev;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The map of unit u: binary search over the maps' first units (entries
// base[0..n], base[n] = all units), the last hit kept.
struct MapOf {
    uint32_t m = 0, lo = 1, hi = 0;
    __device__ __forceinline__ uint32_t find(const uint32_t *base_, uint32_t n, uint32_t u)
    {
        if (u < lo || u >= hi) {
            const CFAR_GLOBAL uint32_t *base = (const CFAR_GLOBAL uint32_t *)base_;
            uint32_t a = 0, b = n;  // base[a] <= u < base[b]
            while (b - a > 1) {
                const uint32_t c = (a + b) >> 1;
                if (uni(base[c]) <= u)
                    a = c;
                else
                    b = c;
            }
            m = a;
            lo = uni(base[a]);
            hi = uni(base[a + 1]);
        }
        return m;
    }
};

// Descriptor of map m in scalar registers (the fields before the padding).
__device__ __forceinline__ void load_desc(const PlainArgs &a, uint32_t m, PlainDesc &d)
{
    if (a.descs) {
        constexpr int kWords = (int)(offsetof(PlainDesc, pad) / 4);
        const CFAR_GLOBAL uint32_t *src = (const CFAR_GLOBAL uint32_t *)(a.descs + m);
        uint32_t w[kWords];
#pragma unroll
        for (int i = 0; i < kWords; ++i) w[i] = uni(src[i]);
        __builtin_memcpy(&d, w, sizeof w);
    } else {
        d = a.single;
    }
}

__device__ __forceinline__ double readlane_f64(double v, uint32_t lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), (int)lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), (int)lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum of one double over the wave (the same value in every lane).
__device__ __forceinline__ double wave_total(double v)
{
    double z15 = 0.0, z31 = 0.0;
    return readlane_f64(wave_scan(v, z15, z31), 63);
}

template <typename T>
__device__ __forceinline__ void to_f64(const T (&v)[kPlainK], double (&x)[kPlainK])
{
#pragma unroll
    for (int k = 0; k < kPlainK; ++k) x[k] = (double)v[k];
}

// Geometry of one integral-image unit.
struct SatUnit {
    int R, F, s, c, r0, r1, jl;
    uint64_t xb, pitch;
    uint32_t xbytes;
    __device__ __forceinline__ SatUnit(const PlainDesc &d, uint32_t local, int lane, int elem)
    {
        R = d.m.rows;
        F = d.m.cols;
        s = (int)(local % (uint32_t)d.n_strips);
        c = (int)(local / (uint32_t)d.n_strips);
        r0 = c * d.chunk;
        r1 = min(r0 + d.chunk, R);
        jl = s * kPlainW + lane * kPlainK;
        xb = (uint64_t)(uintptr_t)d.m.x;
        pitch = (uint64_t)d.m.ld * (uint64_t)elem;
        xbytes = (uint32_t)F * (uint32_t)elem;
    }
    // map row i (r0 <= i < r1): its F elements
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t xrow(int i) const
    {
        return rsrc(xb + (uint64_t)(uint32_t)i * pitch, xbytes);
    }
};

constexpr int kSatPD = 8;  // rows of loads in flight in the integral-image kernels

// plain_aggregate for one unit: left[s][i] = row i summed over the unit's
// columns; V[c][j] = the unit's column totals summed over columns j0..j.
template <typename T>
__device__ __forceinline__ void aggregate_unit(const PlainDesc &d, uint32_t local, int lane)
{
    const SatUnit g(d, local, lane, (int)sizeof(T));
    const uint32_t voff = (uint32_t)g.jl * (uint32_t)sizeof(T);  // columns >= F read zero
    double cs[kPlainK] = {0.0, 0.0, 0.0, 0.0};
    double rt = 0.0;  // lane (i - r0) % 64 holds the total of row i
    double z15 = 0.0, z31 = 0.0;
    T v[kSatPD][kPlainK];
#pragma unroll
    for (int j = 0; j < kSatPD; ++j) ld_row<kPlainK, T>(g.xrow(min(g.r0 + j, g.r1 - 1)), voff, v[j]);
    double *left = d.left + (size_t)g.s * (size_t)g.R;
    for (int i0 = g.r0; i0 < g.r1; i0 += kSatPD) {
#pragma unroll
        for (int j = 0; j < kSatPD; ++j) {
            const int i = i0 + j;
            if (i < g.r1) {  // wave-uniform
                double x[kPlainK];
                to_f64(v[j], x);
                ld_row<kPlainK, T>(g.xrow(min(i + kSatPD, g.r1 - 1)), voff, v[j]);
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < kPlainK; ++k) {
                    cs[k] += x[k];
                    t += x[k];
                }
                const double tot = readlane_f64(wave_scan(t, z15, z31), 63);
                const int q = (i - g.r0) & 63;
                rt = lane == q ? tot : rt;
                if (q == 63 || i == g.r1 - 1) {  // wave-uniform: flush rows i-q .. i
                    if (lane <= q) left[i - q + lane] = rt;
                }
            }
        }
    }
    double p[kPlainK];
    p[0] = cs[0];
#pragma unroll
    for (int k = 1; k < kPlainK; ++k) p[k] = p[k - 1] + cs[k];
    double y15 = 0.0, y31 = 0.0;
    const double ex = wave_scan(p[kPlainK - 1], y15, y31) - p[kPlainK - 1];
    const __amdgpu_buffer_rsrc_t vr =
        rsrc((uint64_t)(uintptr_t)d.V + (uint64_t)(uint32_t)g.c * (uint64_t)g.F * 8u, (uint32_t)g.F * 8u);
#pragma unroll
    for (int k = 0; k < kPlainK; ++k)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, ex + p[k]), vr, (uint32_t)(g.jl + k) * 8u,
                                              0u, 0);
}

// plain_finalize for one unit: S = A + L + V + P (see the top of the file).
template <typename T>
__device__ __forceinline__ void finalize_unit(const PlainDesc &d, uint32_t local, int lane)
{
    const SatUnit g(d, local, lane, (int)sizeof(T));
    const uint32_t voff = (uint32_t)g.jl * (uint32_t)sizeof(T);
    const uint32_t v8 = (uint32_t)g.jl * 8u;
    const double *vrow = d.V + (size_t)g.c * (size_t)g.F;
    // V(c, j) of the lane's columns (zero right of the map)
    double base[kPlainK];
    {
        const __amdgpu_buffer_rsrc_t vr = rsrc((uint64_t)(uintptr_t)vrow, (uint32_t)g.F * 8u);
        ld_row<kPlainK, double>(vr, v8, base);
    }
    // A(c, s): V at the last column of every strip to the left
    double a_part = 0.0;
    for (int s0 = 0; s0 < g.s; s0 += 64) {
        const int t = s0 + lane;
        if (t < g.s) a_part += vrow[min(t * kPlainW + kPlainW - 1, g.F - 1)];
    }
    const double A = wave_total(a_part);
    const double *left = d.left + (size_t)g.s * (size_t)g.R;
    const uint64_t sb = (uint64_t)(uintptr_t)d.S;
    const uint64_t spitch = (uint64_t)g.F * 8u;
    double col[kPlainK] = {0.0, 0.0, 0.0, 0.0};
    double lrun = 0.0, lv = 0.0;
    double z15 = 0.0, z31 = 0.0;
    T v[kSatPD][kPlainK];
#pragma unroll
    for (int j = 0; j < kSatPD; ++j) ld_row<kPlainK, T>(g.xrow(min(g.r0 + j, g.r1 - 1)), voff, v[j]);
    for (int i0 = g.r0; i0 < g.r1; i0 += kSatPD) {
#pragma unroll
        for (int j = 0; j < kSatPD; ++j) {
            const int i = i0 + j;
            if (i < g.r1) {  // wave-uniform
                const int q = (i - g.r0) & 63;
                if (q == 0) {  // the next 64 rows' left carries, one per lane
                    const int r = i + lane;
                    lv = r < g.r1 ? left[r] : 0.0;
                }
                double x[kPlainK];
                to_f64(v[j], x);
                ld_row<kPlainK, T>(g.xrow(min(i + kSatPD, g.r1 - 1)), voff, v[j]);
                double p[kPlainK];
                p[0] = x[0];
#pragma unroll
                for (int k = 1; k < kPlainK; ++k) p[k] = p[k - 1] + x[k];
                const double ex = wave_scan(p[kPlainK - 1], z15, z31) - p[kPlainK - 1];
                lrun += readlane_f64(lv, (uint32_t)q);
                const double al = A + lrun;
                const __amdgpu_buffer_rsrc_t sr = rsrc(sb + (uint64_t)(uint32_t)i * spitch, (uint32_t)spitch);
#pragma unroll
                for (int k = 0; k < kPlainK; k += 2) {
                    col[k] += ex + p[k];
                    col[k + 1] += ex + p[k + 1];
                    double o[2] = {(base[k] + al) + col[k], (base[k + 1] + al) + col[k + 1]};
                    u32x4 w;
                    __builtin_memcpy(&w, o, 16);
                    __builtin_amdgcn_raw_buffer_store_b128(w, sr, v8 + 8u * k, 0u, 0);
                }
            }
        }
    }
}

__global__ void __launch_bounds__(64) plain_aggregate(PlainArgs a)
{
    const int lane = threadIdx.x & 63;
    MapOf mo;
    for (uint32_t u = blockIdx.x; u < a.sat_units; u += gridDim.x) {
        const uint32_t m = a.descs ? mo.find(a.sat_base, a.n_maps, u) : 0u;
        PlainDesc d;
        load_desc(a, m, d);
        const uint32_t local = u - (a.descs ? mo.lo : 0u);
        if (d.m.dtype == 0)
            aggregate_unit<float>(d, local, lane);
        else
            aggregate_unit<double>(d, local, lane);
    }
}

__global__ void __launch_bounds__(64) plain_finalize(PlainArgs a)
{
    const int lane = threadIdx.x & 63;
    MapOf mo;
    for (uint32_t u = blockIdx.x; u < a.sat_units; u += gridDim.x) {
        const uint32_t m = a.descs ? mo.find(a.sat_base, a.n_maps, u) : 0u;
        PlainDesc d;
        load_desc(a, m, d);
        const uint32_t local = u - (a.descs ? mo.lo : 0u);
        if (d.m.dtype == 0)
            finalize_unit<float>(d, local, lane);
        else
            finalize_unit<double>(d, local, lane);
    }
}

// Exclusive scans in place, eight loads in flight: p[0], p[stride], ...
__device__ __forceinline__ void excl_scan_strided(double *p, int n, size_t stride)
{
    double run = 0.0;
    for (int i0 = 0; i0 < n; i0 += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = i0 + q < n ? p[(size_t)(i0 + q) * stride] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (i0 + q < n) p[(size_t)(i0 + q) * stride] = run;
            run += v[q];
        }
    }
}

// Per map: ceil(cols/256) workgroups scan V down the chunks (one column per
// thread), then ceil(rows/256) workgroups scan left across the strips (one
// row per thread).
__global__ void __launch_bounds__(256) plain_carry(PlainArgs a)
{
    MapOf mo;
    const uint32_t b = blockIdx.x;
    const uint32_t m = a.descs ? mo.find(a.blk_base, a.n_maps, b) : 0u;
    PlainDesc d;
    load_desc(a, m, d);
    const uint32_t lb = b - (a.descs ? mo.lo : 0u);
    const int R = d.m.rows, F = d.m.cols;
    const uint32_t nbc = (uint32_t)((F + 255) / 256);
    const int t = (int)threadIdx.x;
    if (lb < nbc) {
        const int j = (int)lb * 256 + t;
        if (j < F) excl_scan_strided(d.V + j, d.n_chunks, (size_t)F);
    } else {
        const int i = (int)(lb - nbc) * 256 + t;
        if (i < R) excl_scan_strided(d.left + i, d.n_strips, (size_t)R);
    }
}

// ---------------------------------------------------------------------------
// Stencil
// ---------------------------------------------------------------------------
template <int K, typename T, bool OUT>
struct StUnit {
    static constexpr int BUF = 64 * K * 8;  // bytes of one published row
    const PlainDesc &d;
    const int lane;
    int R, F, hr, gr, hf, gf;
    int ra, rb;           // output rows of the unit
    int c_lane;           // first column of the lane (may be left of the map)
    uint32_t voff_s;      // lane byte offset into an integral-image row (kOff: left of column 0)
    uint32_t voff_x;      // lane byte offset into a map row (kOff: a lane without outputs)
    uint32_t moff, poff;  // mask byte offsets: full ownership / partial (kOff: none)
    bool part;            // some lane owns only part of its K columns (wave-uniform)
    bool edge;            // the strip holds the map's last column (wave-uniform)
    uint32_t lf, kf;      // lane and element of the map's last column (edge strips)
    double beta_col[K];   // beta on rows without row clipping
    Corner<K> c_oh, c_ol, c_ih, c_il;

    // Band and strip of a unit number (false: a padding unit).
    __device__ __forceinline__ static bool place(const PlainDesc &d, uint32_t local, int &b, int &s)
    {
        if (d.st_xcd) {  // slot x of every 8 goes to strip group x
            const uint32_t per = 8u * (uint32_t)d.st_xcd;
            const uint32_t r = local % per;
            b = (int)(local / per);
            s = (int)((r % 8u) * (uint32_t)d.st_xcd + r / 8u);
        } else {
            b = (int)(local / (uint32_t)d.st_strips);
            s = (int)(local % (uint32_t)d.st_strips);
        }
        return b < d.st_bands && s < d.st_strips;
    }

    __device__ __forceinline__ StUnit(const PlainDesc &d_, int b, int s, int lane_, double *lds)
        : d(d_), lane(lane_)
    {
        R = d.m.rows;
        F = d.m.cols;
        hr = d.m.hr;
        gr = d.m.gr;
        hf = d.m.hf;
        gf = d.m.gf;
        ra = b * d.st_band;
        rb = min(ra + d.st_band, R);
        const int c_out0 = s * d.st_tw;
        const int c_out1 = min(c_out0 + d.st_tw, F);
        const int c0 = c_out0 - d.st_halo;
        c_lane = c0 + lane * K;
        voff_s = c_lane >= 0 ? (uint32_t)c_lane * 8u : kOff;
        const bool own = c_lane >= c_out0 && c_lane < c_out1;
        // the map is read only for the cells under test: lanes without
        // outputs (the halo) read nothing
        voff_x = own ? (uint32_t)c_lane * (uint32_t)sizeof(T) : kOff;
        const bool full = own && c_lane + K <= c_out1;
        moff = full ? (uint32_t)c_lane : kOff;
        poff = own && !full ? (uint32_t)c_lane : kOff;
        part = __builtin_amdgcn_ballot_w64(own && !full) != 0ull;
        const int last = F - 1 - c0;  // position of the map's last column in the strip
        edge = last < 64 * K;
        lf = (uint32_t)(last / K);
        kf = (uint32_t)(last % K);
        const CFAR_GLOBAL double *lut = (const CFAR_GLOBAL double *)d.m.lut;
        // columns whose windows the map does not clip take the full table entry
        const double b_full = lut[d.m.n_full];
        const bool clipped = c_lane - hf < 0 || c_lane + K - 1 + hf > F - 1;
#pragma unroll
        for (int k = 0; k < K; ++k) beta_col[k] = b_full;
        if (clipped) {
#pragma unroll
            for (int k = 0; k < K; ++k) beta_col[k] = lut[nt_of(2 * hr + 1, 2 * gr + 1, k)];
        }
        // wait for those loads here: waiting for them inside the row loop
        // would wait for every row load issued after them
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
        const uint32_t base = (uint32_t)(size_t)(lds_char *)lds;
        c_oh.init(hf, lane, base);
        c_ol.init(-hf - 1, lane, base);
        c_ih.init(gf, lane, base + BUF);
        c_il.init(-gf - 1, lane, base + BUF);
    }

    // training cells of the lane's element k on a row whose clipped outer
    // and guard windows have nro and nri rows
    __device__ __forceinline__ int nt_of(int nro, int nri, int k) const
    {
        const int c = min(max(c_lane + k, 0), F - 1);
        return nro * clip_len(c, hf, F) - nri * clip_len(c, gf, F);
    }

    // integral-image row r (r = -1: the zero row above the map)
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t srow(int r) const
    {
        const bool in = r >= 0;
        return rsrc((uint64_t)(uintptr_t)d.S + (in ? (uint64_t)(uint32_t)r * (uint64_t)F * 8u : 0ull),
                    in ? (uint32_t)F * 8u : 0u);
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t xrow(int i) const
    {
        return rsrc((uint64_t)(uintptr_t)d.m.x + (uint64_t)(uint32_t)i * (uint64_t)d.m.ld * sizeof(T),
                    (uint32_t)F * (uint32_t)sizeof(T));
    }

    struct Rows {
        double a[K], b[K], c[K], e[K];  // rows ro1, ro0 - 1, ri1, ri0 - 1
        T u[K];                          // the cells under test
    };
    __device__ __forceinline__ void load(int i, Rows &w) const
    {
        ld_row<K, double>(srow(min(i + hr, R - 1)), voff_s, w.a);
        ld_row<K, double>(srow(max(i - hr, 0) - 1), voff_s, w.b);
        ld_row<K, double>(srow(min(i + gr, R - 1)), voff_s, w.c);
        ld_row<K, double>(srow(max(i - gr, 0) - 1), voff_s, w.e);
        ld_row<K, T>(xrow(i), voff_x, w.u);
    }

    // positions right of the map take the value at its last column
    __device__ __forceinline__ void clamp_right(double (&v)[K]) const
    {
        double sel = v[0];
#pragma unroll
        for (int k = 1; k < K; ++k) sel = k == (int)kf ? v[k] : sel;
        const double last = readlane_f64(sel, lf);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = c_lane + k >= F ? last : v[k];
    }

    // The window rows summed per column (row corners of eq. 4): outer into
    // po, guard into pi; the cells under test into u.
    __device__ __forceinline__ static void diff(const Rows &w, double (&po)[K], double (&pi)[K], T (&u)[K])
    {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            po[k] = w.a[k] - w.b[k];
            pi[k] = w.c[k] - w.e[k];
            u[k] = w.u[k];
        }
    }

    // Column corners of row i from po / pi, the decision with factors beta,
    // and the stores.
    __device__ __forceinline__ void finish(int i, double (&po)[K], double (&pi)[K], const T (&u)[K],
                                           const double (&beta)[K])
    {
        if (edge) {
            clamp_right(po);
            clamp_right(pi);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            *(lds_double *)(size_t)(c_oh.addr0() + 8 * (k * 64)) = po[k];
            *(lds_double *)(size_t)(c_ih.addr0() + 8 * (k * 64)) = pi[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        auto at = [](uint32_t addr) { return *(const lds_double *)(size_t)addr; };
        double oh[K], ol[K], ih[K], il[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            oh[k] = at(c_oh.addr[k]);
            ol[k] = at(c_ol.addr[k]);
            ih[k] = at(c_ih.addr[k]);
            il[k] = at(c_il.addr[k]);
        }
        uint32_t bits[(K + 3) / 4];
#pragma unroll
        for (int q = 0; q < (K + 3) / 4; ++q) bits[q] = 0u;
        double st[K], thr[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            st[k] = (oh[k] - ol[k]) - (ih[k] - il[k]);
            thr[k] = beta[k] * st[k];  // NaN where N_T = 0 (table entry 0): no detection
            bits[k / 4] |= ((double)u[k] > thr[k]) ? (1u << (8 * (k % 4))) : 0u;
        }
        const __amdgpu_buffer_rsrc_t mrs =
            rsrc((uint64_t)(uintptr_t)d.m.mask + (uint64_t)(uint32_t)i * (uint64_t)d.m.ld_mask, (uint32_t)F);
        if constexpr (K == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(bits[0], mrs, moff, 0u, 0);
        } else {
            const u32x2 bw = {bits[0], bits[1]};
            __builtin_amdgcn_raw_buffer_store_b64(bw, mrs, moff, 0u, 0);
        }
        if (part) {  // wave-uniform: the lane that straddles the map's last column stores bytes
#pragma unroll
            for (int k = 0; k < K; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(bits[k / 4] >> (8 * (k % 4))), mrs,
                                                     poff == kOff ? kOff : poff + (uint32_t)k, 0u, 0);
        }
        if constexpr (OUT) {
            const bool own = moff != kOff || poff != kOff;
            const uint32_t o8 = own ? (uint32_t)c_lane * 8u : kOff;
            const uint64_t orow = (uint64_t)(uint32_t)i * (uint64_t)d.m.ld_mask * 8u;
            if (d.m.train_sum) {
                const __amdgpu_buffer_rsrc_t srs =
                    rsrc((uint64_t)(uintptr_t)d.m.train_sum + orow, (uint32_t)F * 8u);
#pragma unroll
                for (int k = 0; k < K; ++k)
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, st[k]), srs,
                                                          o8 == kOff ? kOff : o8 + 8u * k, 0u, 0);
            }
            if (d.m.thresh) {
                const __amdgpu_buffer_rsrc_t trs = rsrc((uint64_t)(uintptr_t)d.m.thresh + orow, (uint32_t)F * 8u);
                const int nro = min(i + hr, R - 1) - max(i - hr, 0) + 1;
                const int nri = min(i + gr, R - 1) - max(i - gr, 0) + 1;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double t = nt_of(nro, nri, k) > 0 ? thr[k] : INFINITY;
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, t), trs,
                                                          o8 == kOff ? kOff : o8 + 8u * k, 0u, 0);
                }
            }
        }
    }

    // Rows whose windows the map clips (within hr of the top or bottom): one
    // after the other, the factors from the table per cell.
    __device__ __forceinline__ void border_rows(int r0, int r1)
    {
        const CFAR_GLOBAL double *lut = (const CFAR_GLOBAL double *)d.m.lut;
        for (int i = r0; i < r1; ++i) {
            Rows w;
            load(i, w);
            const int nro = min(i + hr, R - 1) - max(i - hr, 0) + 1;
            const int nri = min(i + gr, R - 1) - max(i - gr, 0) + 1;
            double beta[K];
#pragma unroll
            for (int k = 0; k < K; ++k) beta[k] = lut[nt_of(nro, nri, k)];
            double po[K], pi[K];
            T u[K];
            diff(w, po, pi, u);
            finish(i, po, pi, u, beta);
        }
    }

    // Rows [r0, r1) whose windows lie inside the map (factors fixed per
    // column), CFAR_PLAIN_PD rows of loads in flight: a row's slot is refilled
    // with the row PD ahead as soon as its values are taken.  No other load
    // is issued in this loop, so waiting for a slot never waits for later ones.
    __device__ __forceinline__ void interior_rows(int r0, int r1)
    {
        if (r0 >= r1) return;
        constexpr int PD = K == 4 ? CFAR_PLAIN_PD : 2;
        Rows w[PD];
#pragma unroll
        for (int j = 0; j < PD; ++j) load(min(r0 + j, r1 - 1), w[j]);
        for (int i0 = r0; i0 < r1; i0 += PD) {
#pragma unroll
            for (int j = 0; j < PD; ++j) {
                const int i = i0 + j;
                if (i < r1) {  // wave-uniform
                    double po[K], pi[K];
                    T u[K];
                    diff(w[j], po, pi, u);
                    load(min(i + PD, r1 - 1), w[j]);
                    finish(i, po, pi, u, beta_col);
                }
            }
        }
    }

    // Rows [r0, r1) whose windows lie inside the map, in chains of step
    // d = hr - gr: row i + d takes as its guard window's corner rows the
    // outer window's of row i (i+d+gr = i+hr, i+d-hr-1 = i-gr-1), so only
    // two integral-image rows are loaded per row after a chain's first.
    // Rows r0, r0+d, r0+2d, ..., then r0+1, r0+1+d, ...; each step issues
    // the next row's loads before its own work.
    __device__ __forceinline__ void load_chain(int i, Rows &w) const
    {
        ld_row<K, double>(srow(i + hr), voff_s, w.a);
        ld_row<K, double>(srow(i - gr - 1), voff_s, w.e);
        ld_row<K, T>(xrow(i), voff_x, w.u);
    }
    __device__ __forceinline__ void interior_chains(int r0, int r1, int dd)
    {
        Rows w[2];
        load(r0, w[0]);
        int i = r0, t = 0;
        auto step = [&](Rows &cur, Rows &nxt) -> bool {
            const int j = i + dd;
            const bool cont = j < r1;  // wave-uniform: the chain goes on
            const bool more = cont || (t + 1 < dd && r0 + t + 1 < r1);
            if (cont) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    nxt.c[k] = cur.a[k];
                    nxt.b[k] = cur.e[k];
                }
                load_chain(j, nxt);
            } else if (more) {
                load(r0 + t + 1, nxt);
            }
            double po[K], pi[K];
            T u[K];
            diff(cur, po, pi, u);
            finish(i, po, pi, u, beta_col);
            if (!cont) {
                ++t;
                i = r0 + t;
            } else {
                i = j;
            }
            return more;
        };
        for (;;) {
            if (!step(w[0], w[1])) break;
            if (!step(w[1], w[0])) break;
        }
    }

    __device__ __forceinline__ void run()
    {
        const int i0 = min(max(hr, ra), rb);  // first row whose windows the map does not clip
        const int i1 = max(min(R - hr, rb), i0);
        border_rows(ra, i0);
        if (CFAR_PLAIN_CHAIN && hr > gr && i1 - i0 > hr - gr)  // wave-uniform
            interior_chains(i0, i1, hr - gr);
        else
            interior_rows(i0, i1);
        border_rows(i1, rb);
    }
};

template <int K, typename T, bool OUT>
__device__ __forceinline__ void stencil_unit(const PlainDesc &d, uint32_t local, int lane, double *lds)
{
    int b, s;
    if (!StUnit<K, T, OUT>::place(d, local, b, s)) return;
    StUnit<K, T, OUT> w(d, b, s, lane, lds);
    w.run();
}

// Units of maps whose st_k is not K are left to the launch for their K.
template <int K, bool OUT>
__global__ void __launch_bounds__(64) plain_stencil(PlainArgs a)
{
    __shared__ double lds[2 * 64 * K];
    const int lane = threadIdx.x & 63;
    MapOf mo;
    for (uint32_t u = blockIdx.x; u < a.st_units; u += gridDim.x) {
        const uint32_t m = a.descs ? mo.find(a.st_base, a.n_maps, u) : 0u;
        PlainDesc d;
        load_desc(a, m, d);
        if (d.st_k != K) continue;
        const uint32_t local = u - (a.descs ? mo.lo : 0u);
        if (d.m.dtype == 0)
            stencil_unit<K, float, OUT>(d, local, lane, lds);
        else
            stencil_unit<K, double, OUT>(d, local, lane, lds);
    }
}

// Workgroups of one wave that fit the device at once.
int resident_waves(const void *fn, size_t lds)
{
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * prop.multiProcessorCount;
}

}  // namespace

hipError_t launch_plain(const PlainArgs &a, int k_mask, bool with_stencil, bool any_out, hipStream_t stream)
{
    static int g_agg = 0, g_fin = 0;
    if (!g_agg) g_agg = resident_waves((const void *)plain_aggregate, 0);
    if (!g_fin) g_fin = resident_waves((const void *)plain_finalize, 0);
    // a multiple of 8 workgroups where there is room: each wave then stays
    // on the XCD its first unit number maps to (see the stencil's unit order)
    auto grid = [](uint32_t units, int resident) {
        uint32_t g = std::min(units, (uint32_t)resident);
        if (g >= 8) g -= g % 8;
        return dim3(std::max(1u, g));
    };
    hipLaunchKernelGGL(plain_aggregate, grid(a.sat_units, g_agg), dim3(64), 0, stream, a);
    hipLaunchKernelGGL(plain_carry, dim3(std::max(1u, a.carry_blocks)), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(plain_finalize, grid(a.sat_units, g_fin), dim3(64), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !with_stencil || a.st_units == 0) return e;
#define CFAR_ST(K_, O_)                                                                                \
    do {                                                                                               \
        static int g_res = 0;                                                                          \
        if (!g_res) g_res = resident_waves((const void *)plain_stencil<K_, O_>, 0);                   \
        hipLaunchKernelGGL((plain_stencil<K_, O_>), grid(a.st_units, g_res), dim3(64), 0, stream, a); \
    } while (0)
    if (k_mask & 4) {
        if (any_out) CFAR_ST(4, true); else CFAR_ST(4, false);
    }
    if (k_mask & 8) {
        if (any_out) CFAR_ST(8, true); else CFAR_ST(8, false);
    }
#undef CFAR_ST
    return hipGetLastError();
}

}  // namespace cfar
