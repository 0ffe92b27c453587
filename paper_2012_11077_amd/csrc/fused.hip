// TILED CA-CFAR for gfx950: the persistent fused kernel.
//
// Method: Rohman, Andra, Nishimoto, arXiv 2012.11077, Sec. II.B.  The eight
// corners of eq. (4) (outer window minus guard window) are separable: the
// row corners are differences of column prefix sums, the column corners
// differences of row prefixes.  So one pass over the map computes every
// training sum without writing the integral image of eq. (3):
//
//   1. per column of a strip, two FP64 running sums over the rows of the
//      outer window (r-hr .. r+hr) and of the guard window (r-gr .. r+gr):
//      each row step adds the row that enters and takes off the row that
//      leaves, the same FP32 -> FP64 value that was added;
//   2. an FP64 prefix of those column sums along the strip (in-lane over
//      the lane's K columns, then a DPP scan over the 64 lanes), published
//      to LDS;
//   3. the column corners, prefix differences at +h and -h-1, read back;
//   4. S_T = outer - guard, T = beta(N_T) * S_T with beta(N) = alpha(N)/N
//      (eq. 2), decision CUT > T (eq. 1).
//
// One wave per work unit: a strip of W = 64*K columns (lane l holds columns
// cs + l*K .. cs + l*K + K - 1) and a range of output rows of one map.
// Borders cost nothing in the loads: every row is read through a buffer
// resource of its own whose size is the map row (F elements), or zero for a
// row outside the map, so columns right of the map and rows above or below
// it read as zeros (the clipped sums of eq. 4); lanes left of column 0 read
// through an offset past any resource.  Only the threshold factor depends on
// the border: N_T is fixed per column on rows at least hr from the top and
// bottom, and taken per cell from the table on the rest.
#include "internal.h"
#include "devutil.h"

#include <cmath>
#include <type_traits>

// Rows of loads in flight in the interior loop: of the lead row (CFAR_PL)
// and of the other four rows (CFAR_PD) without the guard ring, of the two
// rows still read from memory (CFAR_PDR) with it; waves per SIMD the FP32
// kernel's registers aim at (CFAR_WAVES).  Measured on the uneven batch:
// depth beats occupancy (2 waves per SIMD), and the ring loop gains from
// eight rows of the far rows in flight (2.67 ms against 2.73 ms at four),
// but from only two rows of the lead row in flight (2.334 ms against 2.383
// at four, 2.51 at eight and 2.49 at one).
#ifndef CFAR_PD
#define CFAR_PD 4
#endif
#ifndef CFAR_PL
#define CFAR_PL 2
#endif
#ifndef CFAR_PDR
#define CFAR_PDR 8
#endif
#ifndef CFAR_WAVES
#define CFAR_WAVES 2
#endif
// Guard ring in LDS for the interior rows (when the launch's ring holds it).
#ifndef CFAR_RING
#define CFAR_RING 1
#endif

namespace cfar {

namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// One work unit.
// ---------------------------------------------------------------------------
template <int K, typename T, bool OUT>
struct Unit {
    static constexpr int S = (int)sizeof(T);
    static constexpr int BUF = 64 * K * 8;  // bytes of one prefix row (outer window, then guard window)
    // rows of loads in flight: of the lead row (new data), of the other rows
    static constexpr int PL = K * S >= 32 ? 1 : CFAR_PL;
    static constexpr int PD = K * S >= 32 ? 1 : CFAR_PD;
    static constexpr int PDR = K * S >= 32 ? 1 : CFAR_PDR;  // the ring loop's other rows (two per step)
    static constexpr int U = PL > PD ? PL : PD;      // loop unroll
    static constexpr int UR = PL > PDR ? PL : PDR;   // loop unroll with the ring
    static_assert((PL == 1 || PL == 2 || PL == 4 || PL == 8) && (PD == 1 || PD == 2 || PD == 4 || PD == 8) &&
                      (PDR == 1 || PDR == 2 || PDR == 4 || PDR == 8),
                  "slots rotate by powers of 2");

    const MapDesc &d;
    const int lane;
    int R, F, hr, gr, hf, gf;
    int c_lane;
    int ra, rb;             // output rows of the unit
    int lo, hi;             // map rows the unit reads: [lo, hi]
    uint32_t p32, mp32;     // bytes between map rows, between mask rows
    uint32_t xbytes;        // bytes of a map row's elements
    uint64_t xlo, mra;      // byte addresses of map row lo and of mask row ra
    uint32_t voff;          // lane byte offset into a map row (kOff: left of column 0)
    uint32_t moff;          // lane byte offset of its K mask bytes (kOff: no full ownership)
    uint32_t poff;          // lane byte offset of a partly owned lane (kOff: none)
    uint64_t part;          // lanes that own only part of their K columns (a wave-wide ballot)
    double beta_col[K];     // beta on rows without row clipping
    Corner<K> c_oh, c_ol, c_ih, c_il;
    double Co[K], Ci[K];
    double z15o = 0.0, z31o = 0.0, z15i = 0.0, z31i = 0.0;

    __device__ __forceinline__ Unit(const MapDesc &d_, int strip, int rchunk, int lane_, double *lds_, int ring_off)
        : d(d_), lane(lane_)
    {
        R = d.rows;
        F = d.cols;
        hr = d.hr;
        gr = d.gr;
        hf = d.hf;
        gf = d.gf;
        ra = rchunk * d.rs;
        rb = min(ra + d.rs, R);
        lo = max(ra - hr - 1, 0);
        hi = min(rb - 1 + hr, R - 1);
        const int c_out0 = strip * d.tw;
        const int c_out1 = min(c_out0 + d.tw, F);
        c_lane = c_out0 - d.halo_f + lane * K;
        // row offsets inside the unit's rows fit 32 bits (checked on the host)
        p32 = (uint32_t)d.ld * (uint32_t)S;
        mp32 = (uint32_t)d.ld_mask;
        xbytes = (uint32_t)F * (uint32_t)S;
        xlo = (uint64_t)(uintptr_t)d.x + (uint64_t)(uint32_t)lo * (uint64_t)p32;
        mra = (uint64_t)(uintptr_t)d.mask + (uint64_t)(uint32_t)ra * (uint64_t)mp32;
        voff = c_lane >= 0 ? (uint32_t)c_lane * (uint32_t)S : kOff;
        const bool own = c_lane >= c_out0 && c_lane < c_out1;
        const bool full = own && c_lane + K <= c_out1;
        moff = full ? (uint32_t)c_lane : kOff;
        poff = own && !full ? (uint32_t)c_lane : kOff;
        part = __builtin_amdgcn_ballot_w64(own && !full);
        const CFAR_GLOBAL double *lut = (const CFAR_GLOBAL double *)d.lut;
#pragma unroll
        for (int k = 0; k < K; ++k) beta_col[k] = lut[nt_of(2 * hr + 1, 2 * gr + 1, k)];
        // corner addresses: the outer window's prefix row, then the guard window's
        const uint32_t base = (uint32_t)(size_t)(lds_char *)lds_;
        // the ring after the prefix rows of the launch's largest k
        ring0 = base + (uint32_t)ring_off + (uint32_t)lane * (uint32_t)(K * S);
        asm volatile("" : "+v"(ring0));
        c_oh.init(hf, lane, base);
        c_ol.init(-hf - 1, lane, base);
        c_ih.init(gf, lane, base + BUF);
        c_il.init(-gf - 1, lane, base + BUF);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            Co[k] = 0.0;
            Ci[k] = 0.0;
        }
    }

    // Training cells of the lane's element k on a row whose clipped outer
    // and guard windows have nro and nri rows.
    __device__ __forceinline__ int nt_of(int nro, int nri, int k) const
    {
        const int c = min(max(c_lane + k, 0), F - 1);
        return nro * clip_len(c, hf, F) - nri * clip_len(c, gf, F);
    }

    // Map row i as a buffer resource of its own: its F elements (columns
    // right of the map read zero), or nothing for a row outside the map (its
    // address clamped into the unit's rows).
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t xrow(int i) const
    {
        const uint32_t off = uni((uint32_t)(min(max(i, lo), hi) - lo) * p32);
        return rsrc(xlo + off, (uint32_t)i < (uint32_t)R ? xbytes : 0u);
    }
    // Mask row r as a buffer resource of its F bytes.
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t mrow(int r) const
    {
        return rsrc(mra + uni((uint32_t)(r - ra) * mp32), (uint32_t)F);
    }
    // 1.0 for a row inside the map, else 0.0
    __device__ __forceinline__ static double in_map(int i, int n) { return (uint32_t)i < (uint32_t)n ? 1.0 : 0.0; }

    // Column sums before the first output row ra: Co over rows ra-hr-1 ..
    // ra+hr-1, Ci over rows ra-gr-1 .. ra+gr-1, so that the first step, like
    // every later one, adds rows r+hr, r+gr and takes off rows r-hr-1, r-gr-1.
    // Two batches of rows in flight (the loads of the next batch are issued
    // before the current one is summed); with fill set, the rows of the guard
    // window (ra-gr-1 .. ra+gr-1) also go into the guard ring.
    __device__ __forceinline__ void warm(bool fill)
    {
        constexpr int WB = K * S >= 64 ? 2 : K * S >= 32 ? 4 : 8;
        const int w0 = ra - hr - 1, w1 = ra + hr;  // [w0, w1)
        const int g0 = ra - gr - 1, g1 = ra + gr;
        T v[2][WB][K];
        // rows past w1 - 1 load that row again (a cache hit; never summed)
        auto issue = [&](T (&b)[WB][K], int i0) {
#pragma unroll
            for (int j = 0; j < WB; ++j) ld_row<K, T>(xrow(min(i0 + j, w1 - 1)), voff, b[j]);
        };
        auto take = [&](const T (&b)[WB][K], int i0) {
#pragma unroll
            for (int j = 0; j < WB; ++j) {
                const int i = i0 + j;
                const bool guard = i >= g0 && i < g1;  // wave-uniform
                const double wo = i < w1 ? in_map(i, R) : 0.0;
                const double wi = guard ? wo : 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    Co[k] = __builtin_fma(wo, (double)b[j][k], Co[k]);
                    Ci[k] = __builtin_fma(wi, (double)b[j][k], Ci[k]);
                }
                if (fill && guard) ring_put(ring_slot(i), b[j]);
            }
        };
        issue(v[0], w0);
        for (int i0 = w0; i0 < w1; i0 += 2 * WB) {
            issue(v[1], i0 + WB);
            take(v[0], i0);
            issue(v[0], i0 + 2 * WB);
            take(v[1], i0 + WB);
        }
    }

    // The loads of row step r other than the lead row r+hr: rows r+gr,
    // r-gr-1, r-hr-1 and the cells under test (row r).
    struct Rest {
        T b[K], c[K], e[K], u[K];
    };
    __device__ __forceinline__ void load_lead(int r, T (&a)[K]) const { ld_row<K, T>(xrow(r + hr), voff, a); }
    __device__ __forceinline__ void load_rest(int r, Rest &s) const
    {
        ld_row<K, T>(xrow(r + gr), voff, s.b);
        ld_row<K, T>(xrow(r - gr - 1), voff, s.c);
        ld_row<K, T>(xrow(r - hr - 1), voff, s.e);
        ld_row<K, T>(xrow(r), voff, s.u);
    }

    // Running column sums for row r, then the strip prefix of both into LDS.
    // Rows outside the map read as zeros, so adding and taking them off
    // leaves the sums as they are.  (One buffer per window: a wave's LDS
    // operations complete in order, so the corner reads of a row are done
    // before the next row's writes.)
    __device__ __forceinline__ void accumulate_publish(const T (&a)[K], const Rest &s)
    {
        accumulate_publish(a, s.b, s.c, s.e);
    }
    __device__ __forceinline__ void accumulate_publish(const T (&a)[K], const T (&b)[K], const T (&c)[K],
                                                       const T (&e)[K])
    {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            Co[k] = (Co[k] + (double)a[k]) - (double)e[k];
            Ci[k] = (Ci[k] + (double)b[k]) - (double)c[k];
        }
        double po[K], pi[K];
        po[0] = Co[0];
        pi[0] = Ci[0];
#pragma unroll
        for (int k = 1; k < K; ++k) {
            po[k] = po[k - 1] + Co[k];
            pi[k] = pi[k - 1] + Ci[k];
        }
        // exclusive prefix of the lane totals: the inclusive one minus the lane's own
        const double eo = wave_scan(po[K - 1], z15o, z31o) - po[K - 1];
        const double ei = wave_scan(pi[K - 1], z15i, z31i) - pi[K - 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            *(lds_double *)(size_t)(c_oh.addr0() + 8 * (k * 64)) = eo + po[k];
            *(lds_double *)(size_t)(c_ih.addr0() + 8 * (k * 64)) = ei + pi[k];
        }
        // LDS operations of one wave complete in order; keep the compiler from
        // moving the corner reads that follow above these writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // The four column corners of every cell of the lane.
    struct Corners {
        double oh[K], ol[K], ih[K], il[K];
    };
    __device__ __forceinline__ void corners(Corners &c) const
    {
        auto at = [](uint32_t a) { return *(const lds_double *)(size_t)a; };
#pragma unroll
        for (int k = 0; k < K; ++k) {
            c.oh[k] = at(c_oh.addr[k]);
            c.ol[k] = at(c_ol.addr[k]);
            c.ih[k] = at(c_ih.addr[k]);
            c.il[k] = at(c_il.addr[k]);
        }
    }

    // eqs. (1), (2), (4) for the lane's K cells of row r with factors beta,
    // and the stores.
    __device__ __forceinline__ void decide(int r, const Corners &c, const T (&u)[K], const double (&beta)[K])
    {
        decide(r, c, u, beta, mrow(r));
    }
    __device__ __forceinline__ void decide(int r, const Corners &c, const T (&u)[K], const double (&beta)[K],
                                           __amdgpu_buffer_rsrc_t mrs)
    {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        uint32_t bits[(K + 3) / 4];
#pragma unroll
        for (int q = 0; q < (K + 3) / 4; ++q) bits[q] = 0u;
        double st[K], thr[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            st[k] = (c.oh[k] - c.ol[k]) - (c.ih[k] - c.il[k]);
            thr[k] = beta[k] * st[k];  // NaN where N_T = 0 (table entry 0): no detection
            bits[k / 4] |= ((double)u[k] > thr[k]) ? (1u << (8 * (k % 4))) : 0u;
        }
        const uint32_t ms = 0u;
        if constexpr (K == 2) {
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)bits[0], mrs, moff, ms, 0);
        } else if constexpr (K == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(bits[0], mrs, moff, ms, 0);
        } else {
            const u32x2 w = {bits[0], bits[1]};
            __builtin_amdgcn_raw_buffer_store_b64(w, mrs, moff, ms, 0);
        }
        uint64_t pf = part;
        asm volatile("" : "+s"(pf));  // a scalar branch, not a lane mask
        if (pf != 0ull) {  // wave-uniform: the lane that straddles the map's last column stores bytes
#pragma unroll
            for (int k = 0; k < K; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(bits[k / 4] >> (8 * (k % 4))), mrs,
                                                     poff == kOff ? kOff : poff + (uint32_t)k, ms, 0);
        }
        if constexpr (OUT) {
            const bool own = moff != kOff || poff != kOff;
            const uint32_t o8 = own ? (uint32_t)c_lane * 8u : kOff;
            const int nro = clip_len(r, hr, R), nri = clip_len(r, gr, R);
            const uint64_t orow = (uint64_t)(uint32_t)r * (uint64_t)d.ld_mask * 8u;
            if (d.train_sum) {
                const __amdgpu_buffer_rsrc_t srs = rsrc((uint64_t)(uintptr_t)d.train_sum + orow, (uint32_t)F * 8u);
#pragma unroll
                for (int k = 0; k < K; ++k)
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, st[k]), srs,
                                                          o8 == kOff ? kOff : o8 + 8u * k, 0u, 0);
            }
            if (d.thresh) {
                const __amdgpu_buffer_rsrc_t trs = rsrc((uint64_t)(uintptr_t)d.thresh + orow, (uint32_t)F * 8u);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double t = nt_of(nro, nri, k) > 0 ? thr[k] : INFINITY;
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, t), trs,
                                                          o8 == kOff ? kOff : o8 + 8u * k, 0u, 0);
                }
            }
        }
    }
    // Rows [r, r1) through f(slot, row), slots 0..U-1 in turn: full rounds of
    // U rows, then the remaining rows of a last round.
    template <int UU, typename Fn>
    __device__ __forceinline__ void unrolled_rows(int r, int r1, Fn &f)
    {
        for (; r + UU <= r1; r += UU) round<0, UU>(r, r1, f);
        round<0, UU>(r, r1, f);  // < UU rows left
    }
    template <int J, int UU, typename Fn>
    __device__ __forceinline__ void round(int r, int r1, Fn &f)
    {
        if constexpr (J < UU) {
            if (r + J < r1) {  // wave-uniform; always true in full rounds
                f(std::integral_constant<int, J>(), r + J);
                round<J + 1, UU>(r, r1, f);
            }
        }
    }

    // Rows whose windows the map clips (within hr of the top or bottom):
    // one after the other, the factors from the table per cell.
    __device__ __forceinline__ void border_rows(int r0, int r1)
    {
        for (int r = r0; r < r1; ++r) {
            T a[K];
            Rest s;
            load_lead(r, a);
            load_rest(r, s);
            const int nro = clip_len(r, hr, R), nri = clip_len(r, gr, R);
            const CFAR_GLOBAL double *lut = (const CFAR_GLOBAL double *)d.lut;
            double beta[K];
#pragma unroll
            for (int k = 0; k < K; ++k) beta[k] = lut[nt_of(nro, nri, k)];
            accumulate_publish(a, s);
            Corners c;
            corners(c);
            decide(r, c, s.u, beta);
        }
    }

    // One row of the interior loop, slot J: the lead row's loads run PL rows
    // ahead, the other rows' PD rows; rows past the end are clamped to the
    // last (loaded again, harmless).
    template <int J>
    __device__ __forceinline__ void irow(int r, int r1, T (&lead)[PL][K], Rest (&rest)[PD])
    {
        constexpr int JL = J % PL, JR = J % PD;
        accumulate_publish(lead[JL], rest[JR]);
        T u[K];
#pragma unroll
        for (int k = 0; k < K; ++k) u[k] = rest[JR].u[k];
        load_lead(min(r + PL, r1 - 1), lead[JL]);
        load_rest(min(r + PD, r1 - 1), rest[JR]);
        Corners c;
        corners(c);
        decide(r, c, u, beta_col);
    }

    // Rows [r0, r1) whose windows lie inside the map: factors fixed per column.
    __device__ __forceinline__ void interior_rows(int r0, int r1)
    {
        if (r0 >= r1) return;
        T lead[PL][K];
        Rest rest[PD];
#pragma unroll
        for (int j = 0; j < PL; ++j) load_lead(min(r0 + j, r1 - 1), lead[j]);
#pragma unroll
        for (int j = 0; j < PD; ++j) load_rest(min(r0 + j, r1 - 1), rest[j]);
        int r = r0;
        auto one = [&](auto jt, int rr) { irow<decltype(jt)::value>(rr, r1, lead, rest); };
        unrolled_rows<U>(r, r1, one);
    }

    // The guard ring: the rows r-gr-1 .. r+gr of the strip in LDS (slot of
    // row i: i mod D, D = 2gr+2), each lane's K values at lane*K*S.  Row r+gr
    // comes from global memory and goes into the ring; rows r (the cells
    // under test) and r-gr-1 (leaving the guard window) come back from it, so
    // a row step loads three rows instead of five.
    struct RestR {
        T b[K], e[K];
    };
    static constexpr uint32_t RROW = 64u * K * S;  // bytes of one ring row
    uint32_t ring0;  // LDS byte address of the lane's values in ring slot 0
    int D;           // ring slots
    __device__ __forceinline__ void ring_put(int slot, const T (&v)[K]) const
    {
        typedef uint32_t r32x4 __attribute__((ext_vector_type(4)));
        const uint32_t a = ring0 + (uint32_t)slot * RROW;
#pragma unroll
        for (int q = 0; q < (int)(K * S / 16); ++q) {
            r32x4 w;
            __builtin_memcpy(&w, (const char *)v + 16 * q, 16);
            *(__attribute__((address_space(3))) r32x4 *)(size_t)(a + 16u * q) = w;
        }
        if constexpr (K * S == 8) *(__attribute__((address_space(3))) uint64_t *)(size_t)a = __builtin_bit_cast(uint64_t, v);
    }
    __device__ __forceinline__ void ring_get(int slot, T (&v)[K]) const
    {
        typedef uint32_t r32x4 __attribute__((ext_vector_type(4)));
        const uint32_t a = ring0 + (uint32_t)slot * RROW;
#pragma unroll
        for (int q = 0; q < (int)(K * S / 16); ++q) {
            const r32x4 w = *(const __attribute__((address_space(3))) r32x4 *)(size_t)(a + 16u * q);
            __builtin_memcpy((char *)v + 16 * q, &w, 16);
        }
        if constexpr (K * S == 8) {
            const uint64_t w = *(const __attribute__((address_space(3))) uint64_t *)(size_t)a;
            __builtin_memcpy(v, &w, 8);
        }
    }
    __device__ __forceinline__ void load_rest(int r, RestR &s) const
    {
        ld_row<K, T>(xrow(r + gr), voff, s.b);
        ld_row<K, T>(xrow(r - hr - 1), voff, s.e);
    }
    // The ring's part of row step r: row r+gr (b) into its slot, the cells
    // under test (row r) and row r-gr-1 out of theirs; the slots move on.
    __device__ __forceinline__ void ring_step(const T (&b)[K], T (&u)[K], T (&c)[K], int &sb, int &su, int &sc)
    {
        ring_put(sb, b);
        // the reads below must see that write (the same slot when gr = 0)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        ring_get(su, u);
        ring_get(sc, c);
        sb = sb + 1 == D ? 0 : sb + 1;
        su = su + 1 == D ? 0 : su + 1;
        sc = sc + 1 == D ? 0 : sc + 1;
    }
    template <int J>
    __device__ __forceinline__ void irow_ring(int r, int r1, T (&lead)[PL][K], RestR (&rest)[PDR], int &sb, int &su,
                                              int &sc)
    {
        constexpr int JL = J % PL, JR = J % PDR;
        T u[K], c[K];
        ring_step(rest[JR].b, u, c, sb, su, sc);
        accumulate_publish(lead[JL], rest[JR].b, c, rest[JR].e);
        load_lead(min(r + PL, r1 - 1), lead[JL]);
        load_rest(min(r + PDR, r1 - 1), rest[JR]);
        Corners cr;
        corners(cr);
        decide(r, cr, u, beta_col);
    }
    // Byte addresses of the rows the next fast step loads (lead row, rows
    // r+gr and r-hr-1) and of its mask row; each step moves all four down a
    // row.
    struct Rows {
        uint64_t l, b, e, m;
    };
    // One row of the ring loop where no load needs clamping (every row it
    // loads lies in the unit's rows and in the map): the row resources come
    // from addresses that move by a row per step instead of being rebuilt
    // from the row index.
    template <int J>
    __device__ __forceinline__ void irow_ring_fast(int r, T (&lead)[PL][K], RestR (&rest)[PDR], int &sb, int &su,
                                                   int &sc, Rows &w)
    {
        constexpr int JL = J % PL, JR = J % PDR;
        T u[K], c[K];
        ring_step(rest[JR].b, u, c, sb, su, sc);
        accumulate_publish(lead[JL], rest[JR].b, c, rest[JR].e);
        ld_row<K, T>(rsrc(w.l, xbytes), voff, lead[JL]);
        ld_row<K, T>(rsrc(w.b, xbytes), voff, rest[JR].b);
        ld_row<K, T>(rsrc(w.e, xbytes), voff, rest[JR].e);
        w.l += p32;
        w.b += p32;
        w.e += p32;
        Corners cr;
        corners(cr);
        decide(r, cr, u, beta_col, rsrc(w.m, (uint32_t)F));
        w.m += mp32;
    }
    // Rows r0-gr-1 .. r0+gr-1 into the guard ring, four loads in flight.
    __device__ __forceinline__ void fill_ring(int r0)
    {
        for (int i0 = r0 - gr - 1; i0 < r0 + gr; i0 += 4) {
            T v[4][K];
#pragma unroll
            for (int j = 0; j < 4; ++j) ld_row<K, T>(xrow(min(i0 + j, r0 + gr - 1)), voff, v[j]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (i0 + j < r0 + gr) ring_put(ring_slot(i0 + j), v[j]);
        }
    }
    __device__ __forceinline__ int ring_slot(int i) const { return (i % D + D) % D; }
    // filled: the ring already holds rows r0-gr-1 .. r0+gr-1 (from warm()).
    __device__ __forceinline__ void interior_rows_ring(int r0, int r1, bool filled)
    {
        if (r0 >= r1) return;
        if (!filled) fill_ring(r0);
        T lead[PL][K];
        RestR rest[PDR];
#pragma unroll
        for (int j = 0; j < PL; ++j) load_lead(min(r0 + j, r1 - 1), lead[j]);
#pragma unroll
        for (int j = 0; j < PDR; ++j) load_rest(min(r0 + j, r1 - 1), rest[j]);
        int sb = (r0 + gr) % D, su = r0 % D, sc = (r0 - gr - 1 + D) % D;
        int r = r0;
        // Steps whose loads (up to PL and PDR rows ahead) stay below r1 need
        // no clamping: rows r+hr+PL <= r1-1+hr and r-hr-1+PDR >= 0 (r >= hr)
        // lie in the unit's rows and in the map.
        constexpr int PM = PL > PDR ? PL : PDR;
        if (r + UR + PM <= r1) {
            Rows w;
            w.l = xlo + (uint64_t)((uint32_t)(r + PL + hr - lo) * p32);
            w.b = xlo + (uint64_t)((uint32_t)(r + PDR + gr - lo) * p32);
            w.e = xlo + (uint64_t)((uint32_t)(r + PDR - hr - 1 - lo) * p32);
            w.m = mra + (uint64_t)((uint32_t)(r - ra) * mp32);
            auto fast = [&](auto jt, int rr) { irow_ring_fast<decltype(jt)::value>(rr, lead, rest, sb, su, sc, w); };
            for (; r + UR + PM <= r1; r += UR) round<0, UR>(r, r1, fast);
        }
        auto one = [&](auto jt, int rr) { irow_ring<decltype(jt)::value>(rr, r1, lead, rest, sb, su, sc); };
        unrolled_rows<UR>(r, r1, one);
    }

    __device__ __forceinline__ void run(int ring_bytes)
    {
        const int i0 = min(max(hr, ra), rb);  // first row whose windows the map does not clip
        const int i1 = max(min(R - hr, rb), i0);
        D = 2 * gr + 2;
        const bool ring = CFAR_RING && i0 < i1 && (uint32_t)D * RROW <= (uint32_t)ring_bytes;  // wave-uniform
        warm(ring && i0 == ra);
        border_rows(ra, i0);
        if (ring)
            interior_rows_ring(i0, i1, i0 == ra);
        else
            interior_rows(i0, i1);
        border_rows(i1, rb);
    }
};

// Waves per SIMD the register allocation aims at.
template <int KS, typename T, bool OUT>
constexpr int fused_waves()
{
    return KS == 8 ? 1 : (sizeof(T) == 4 && !OUT) ? CFAR_WAVES : 2;
}

// One wave per workgroup; dynamic LDS per wave: the outer and the guard
// prefix row, 64*KM doubles each.  KS = 24: each unit runs
// with its map's k (2 or 4); KS = 8: k = 8.
template <int KS, typename T, bool OUT>
__global__ void __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(fused_waves<KS, T, OUT>())))
fused_kernel(FusedArgs args)
{
    extern __shared__ double fused_lds[];
    const int lane = threadIdx.x & 63;
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = __hip_atomic_fetch_add(args.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u = uni(u);
        if (u >= args.total_units) break;
        // descriptor and unit tables are wave-uniform: scalar loads
        uint32_t local = u;
        MapDesc d;
        if (args.descs) {
            const uint32_t m = uni(((const CFAR_GLOBAL uint32_t *)args.unit_map)[u]);
            local = u - uni(((const CFAR_GLOBAL uint32_t *)args.unit_base)[m]);
            const CFAR_GLOBAL uint32_t *src = (const CFAR_GLOBAL uint32_t *)(args.descs + m);
            uint32_t w[sizeof(MapDesc) / 4];
#pragma unroll
            for (int i = 0; i < (int)(sizeof(MapDesc) / 4); ++i) w[i] = uni(src[i]);  // keep it in SGPRs
            __builtin_memcpy(&d, w, sizeof(MapDesc));
        } else {
            d = args.single;
        }
        const int strip = (int)(local % (uint32_t)d.n_strips);
        const int rchunk = (int)(local / (uint32_t)d.n_strips);
        constexpr int KM = KS == 8 ? 8 : 4;
        constexpr int ring_off = 2 * KM * 64 * 8;  // after the two prefix rows
        if constexpr (KS == 8) {
            Unit<8, T, OUT> w(d, strip, rchunk, lane, fused_lds, ring_off);
            w.run(args.ring_bytes);
        } else {
            if (d.k_cols == 2) {
                Unit<2, T, OUT> w(d, strip, rchunk, lane, fused_lds, ring_off);
                w.run(args.ring_bytes);
            } else {
                Unit<4, T, OUT> w(d, strip, rchunk, lane, fused_lds, ring_off);
                w.run(args.ring_bytes);
            }
        }
    }
}

#define CFAR_FUSED_VARIANTS(X_)                                                                        \
    X_(24, float, false) X_(24, float, true) X_(24, double, false) X_(24, double, true)                 \
    X_(8, float, false) X_(8, float, true) X_(8, double, false) X_(8, double, true)

const void *fused_fn(int kset, int dtype, bool out)
{
#define CFAR_PICK(K_, T_, O_)                                             \
    if (kset == K_ && dtype == (sizeof(T_) == 4 ? 0 : 1) && out == O_) \
        return (const void *)fused_kernel<K_, T_, O_>;
    CFAR_FUSED_VARIANTS(CFAR_PICK)
#undef CFAR_PICK
    return nullptr;
}

}  // namespace

int fused_resident_blocks(int kset, int dtype, bool out, int ring_bytes)
{
    // cache: device x kernel x ring size (in 512-byte steps)
    constexpr int kDev = 16, kSteps = 129;
    static int cached[kDev][8][kSteps] = {{{0}}};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    const int slot = ((kset == 8 ? 1 : 0) * 2 + dtype) * 2 + (out ? 1 : 0);
    const int step = ring_bytes % 512 == 0 && ring_bytes / 512 < kSteps ? ring_bytes / 512 : -1;
    int *c = dev < kDev && step >= 0 ? &cached[dev][slot][step] : nullptr;
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
