// Device-side helpers shared by the gate-sweep sources (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include <vector>

#include "sv.h"

namespace sv {
namespace dev {

constexpr int kThreads = 256;
constexpr int kMaxIns = SV_MAX_TARGETS + SV_MAX_CONTROLS;

template <typename R>
struct CT;
template <>
struct CT<float> {
    using C = float2;
};
template <>
struct CT<double> {
    using C = double2;
};

// Insert a 0 bit at each of up to kMaxIns sorted positions: m[j] = 2^p_j - 1.
struct InsertMasks {
    uint64_t m[kMaxIns];
    int n;
};

inline InsertMasks make_insert_masks(std::vector<int> pos)
{
    std::sort(pos.begin(), pos.end());
    InsertMasks im{};
    im.n = static_cast<int>(pos.size());
    for (int j = 0; j < im.n; ++j)
        im.m[j] = (uint64_t(1) << pos[j]) - 1;
    return im;
}

__host__ __device__ __forceinline__ uint64_t insert_zeros(uint64_t g, const InsertMasks &im)
{
    for (int j = 0; j < im.n; ++j) {
        const uint64_t lo = im.m[j];
        g = (g & lo) | ((g & ~lo) << 1);
    }
    return g;
}

template <typename C>
__device__ __forceinline__ C cmad(C u, C v, C acc)
{
    acc.x += u.x * v.x - u.y * v.y;
    acc.y += u.x * v.y + u.y * v.x;
    return acc;
}

template <typename C>
__device__ __forceinline__ C cmul(C u, C v)
{
    C r;
    r.x = u.x * v.x - u.y * v.y;
    r.y = u.x * v.y + u.y * v.x;
    return r;
}

template <typename C>
__device__ __forceinline__ C czero()
{
    C r;
    r.x = 0;
    r.y = 0;
    return r;
}

// LDS address swizzle: low 6 bits ^= next 6 bits.  A bijection on any power
// of two >= 64; lanes that read with a power-of-two stride land on distinct
// banks.
__device__ __forceinline__ uint32_t swz(uint32_t x)
{
    return x ^ ((x >> 6) & 63u);
}

// The same without touching bit 0 (bits 7..11 into bits 1..5): an amplitude
// pair (2m, 2m + 1) stays adjacent and in order, so a tile sweep moves it as
// one 16-byte LDS access.  Also linear over XOR and its own inverse.
__device__ __forceinline__ uint32_t swz_p(uint32_t x)
{
    return x ^ ((x >> 6) & 62u);
}

// Geometry of one LDS tile: the amplitudes spanned by the k target bits and
// the m lowest free bits, for one value of all other bits.  Tile-local index
// x lists the tile bits in ascending physical order.
struct TileArgs {
    uint64_t ntiles;
    uint64_t cmask;
    InsertMasks outer;                 // zeros at tile bits and control bits
    uint64_t dep[13];                  // dep[b] = 2^(physical position of tile bit b)
    uint32_t tslot_m[SV_MAX_TARGETS];  // insert masks of the target slots in x
    int ntslot;
    uint16_t xc[64];                   // x bits of target-row index r
    const void *U;
};

// Fill TileArgs for a k-target block with c controls and 2^ta_log-amplitude
// tiles.  Requires n - c - k >= ta_log - k.
inline TileArgs make_tile_args(int n, int k, const int *tgt, const int *ctl, int c, int ta_log,
                               const void *d_U)
{
    TileArgs a{};
    const int m = ta_log - k;
    uint64_t used = 0;
    for (int b = 0; b < k; ++b)
        used |= uint64_t(1) << tgt[b];
    for (int j = 0; j < c; ++j)
        used |= uint64_t(1) << ctl[j];
    std::vector<int> tilebits(tgt, tgt + k);
    for (int p = 0, got = 0; got < m && p < n; ++p) {
        if (!((used >> p) & 1)) {
            tilebits.push_back(p);
            ++got;
        }
    }
    std::sort(tilebits.begin(), tilebits.end());
    for (int b = 0; b < ta_log; ++b)
        a.dep[b] = uint64_t(1) << tilebits[b];
    int slot[SV_MAX_TARGETS];
    for (int b = 0; b < k; ++b)
        slot[b] = int(std::find(tilebits.begin(), tilebits.end(), tgt[b]) - tilebits.begin());
    std::vector<int> sorted_slots(slot, slot + k);
    std::sort(sorted_slots.begin(), sorted_slots.end());
    a.ntslot = k;
    for (int b = 0; b < k; ++b)
        a.tslot_m[b] = (1u << sorted_slots[b]) - 1u;
    for (int r = 0; r < (1 << k); ++r) {
        uint32_t x = 0;
        for (int b = 0; b < k; ++b)
            if ((r >> b) & 1)
                x |= 1u << slot[b];
        a.xc[r] = uint16_t(x);
    }
    std::vector<int> outer(tilebits.begin(), tilebits.end());
    outer.insert(outer.end(), ctl, ctl + c);
    a.outer = make_insert_masks(outer);
    for (int j = 0; j < c; ++j)
        a.cmask |= uint64_t(1) << ctl[j];
    a.ntiles = uint64_t(1) << (n - c - ta_log);
    a.U = d_U;
    return a;
}

// x-slot of group g: insert zeros at the target slots.
__device__ __forceinline__ uint32_t group_slot(uint32_t g, const TileArgs &a)
{
    for (int s = 0; s < a.ntslot; ++s) {
        const uint32_t lo = a.tslot_m[s];
        g = (g & lo) | ((g & ~lo) << 1);
    }
    return g;
}

// Global offset of tile-local index s * kThreads + tid (low 8 bits from tid).
__device__ __forceinline__ uint64_t tile_low_offset(int tid, const TileArgs &a)
{
    uint64_t off = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((tid >> b) & 1)
            off |= a.dep[b];
    return off;
}

// ---------------------------------------------------------------------------
// Streaming global access.  State sweeps touch every byte exactly once, so
// loads and stores carry the nontemporal hint: lines are not kept in L2 or
// the memory-side cache for reuse that never comes.
// ---------------------------------------------------------------------------
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 ld_nt(const float2 *p)
{
    const f32x2 q = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(p));
    return make_float2(q.x, q.y);
}
__device__ __forceinline__ double2 ld_nt(const double2 *p)
{
    const f64x2 q = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
    return make_double2(q.x, q.y);
}
__device__ __forceinline__ float4 ld_nt(const float4 *p)
{
    const f32x4 q = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
    return make_float4(q.x, q.y, q.z, q.w);
}
__device__ __forceinline__ void st_nt(float2 *p, float2 v)
{
    __builtin_nontemporal_store(f32x2{v.x, v.y}, reinterpret_cast<f32x2 *>(p));
}
__device__ __forceinline__ void st_nt(double2 *p, double2 v)
{
    __builtin_nontemporal_store(f64x2{v.x, v.y}, reinterpret_cast<f64x2 *>(p));
}
__device__ __forceinline__ void st_nt(float4 *p, float4 v)
{
    __builtin_nontemporal_store(f32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<f32x4 *>(p));
}

// ---------------------------------------------------------------------------
// Sweep over LDS tiles, one tile per workgroup: load (all of the
// workgroup's global loads in flight at once) -> LDS -> compute -> store.
// Latency is hidden by the other resident workgroups of the CU rather than by
// a register prefetch of the next tile, which keeps register use low and
// residency high.  The grid is 2-D (tile = blockIdx.y * gridDim.x +
// blockIdx.x, see tile_grid) so that no workgroup loops: a loop would let the
// compiler hoist the per-tile constants into registers.  PAIR (complex64
// with physical bit 0 inside the tile) moves amplitude pairs as 16-byte
// accesses.  NTH is the workgroup size (256 or 512 threads); REMAT
// recomputes the store addresses after compute() instead of keeping them;
// PSWZ lays the tile out with swz_p (pairs as 16-byte LDS accesses; the
// tile must then be 16-byte aligned and compute() must use swz_p).
//
// compute(tile) starts after a barrier that follows the tile's LDS writes; it
// must leave its results in the same LDS slots and end with __syncthreads().
// src(x) (identity by default) is the tile-local index whose LDS slot the
// store of element x reads: a permutation of the tile applied on the way out
// (not with PSWZ).
// ---------------------------------------------------------------------------
struct SameSlot {
    __device__ __forceinline__ uint32_t operator()(uint32_t x) const { return x; }
};

template <typename R, int TA_LOG, bool PAIR, int NTH = kThreads, bool REMAT = false, bool PSWZ = false, typename F,
          typename S = SameSlot>
__device__ __forceinline__ void tile_sweep(R *__restrict__ st, const TileArgs &a, typename CT<R>::C *tile,
                                           F &&compute, S src = S())
{
    using C = typename CT<R>::C;
    constexpr int TA = 1 << TA_LOG;
    constexpr int OPT = TA / NTH;
    constexpr int TB = NTH == 512 ? 9 : 8;  // thread index bits
    static_assert(NTH == 256 || NTH == 512, "256 or 512 threads");
    static_assert(OPT >= 2 && OPT % 2 == 0, "tile smaller than two elements per thread");
    static_assert(!PAIR || std::is_same<R, float>::value, "16-byte pairs are complex64 only");
    constexpr int LO = PAIR ? 1 : 0;  // tile bits below the thread bits
    const int tid = threadIdx.x;
    uint64_t off_lo = 0;
#pragma unroll
    for (int b = 0; b < TB; ++b)
        if ((tid >> b) & 1)
            off_lo |= a.dep[b + LO];
    auto offset = [&](int s) -> uint64_t {
        uint64_t off = off_lo;
#pragma unroll
        for (int b = TB + LO; b < TA_LOG; ++b)
            if ((s >> (b - TB - LO)) & 1)
                off |= a.dep[b];
        return off;
    };
    const uint64_t o = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    if (o >= a.ntiles)
        return;
    const uint64_t base = insert_zeros(o, a.outer) | a.cmask;
    {
        if constexpr (PAIR) {
            const float4 *v4 = reinterpret_cast<const float4 *>(st);
            float4 q[OPT / 2];
#pragma unroll
            for (int s = 0; s < OPT / 2; ++s)
                q[s] = ld_nt(&v4[(base + offset(s)) >> 1]);
#pragma unroll
            for (int s = 0; s < OPT / 2; ++s) {
                const uint32_t x = 2u * uint32_t(s * NTH + tid);
                if constexpr (PSWZ) {
                    *reinterpret_cast<float4 *>(&tile[swz_p(x)]) = q[s];
                } else {
                    tile[swz(x)] = make_float2(q[s].x, q[s].y);
                    tile[swz(x + 1)] = make_float2(q[s].z, q[s].w);
                }
            }
        } else {
            const C *v = reinterpret_cast<const C *>(st);
            R qr[OPT], qi[OPT];  // scalar arrays: vector-typed ones go to scratch
#pragma unroll
            for (int s = 0; s < OPT; ++s) {
                const C q = ld_nt(&v[base + offset(s)]);
                qr[s] = q.x;
                qi[s] = q.y;
            }
#pragma unroll
            for (int s = 0; s < OPT; ++s) {
                C q;
                q.x = qr[s];
                q.y = qi[s];
                tile[PSWZ ? swz_p(uint32_t(s * NTH + tid)) : swz(uint32_t(s * NTH + tid))] = q;
            }
        }
        __syncthreads();
        compute(tile);
        // REMAT: the store addresses are recomputed from a copy of the thread
        // index the compiler cannot see through (an empty asm), so they are
        // not held in registers, or spilled, across a register-hungry
        // compute().
        int tid2 = tid;
        if constexpr (REMAT)
            asm volatile("" : "+v"(tid2));
        uint64_t off_lo2 = 0;
#pragma unroll
        for (int b = 0; b < TB; ++b)
            if ((tid2 >> b) & 1)
                off_lo2 |= a.dep[b + LO];
        auto offset2 = [&](int s) -> uint64_t {
            uint64_t off = off_lo2;
#pragma unroll
            for (int b = TB + LO; b < TA_LOG; ++b)
                if ((s >> (b - TB - LO)) & 1)
                    off |= a.dep[b];
            return off;
        };
        if constexpr (PAIR) {
            float4 *v4 = reinterpret_cast<float4 *>(st);
#pragma unroll
            for (int s = 0; s < OPT / 2; ++s) {
                const uint32_t x = 2u * uint32_t(s * NTH + tid2);
                if constexpr (PSWZ) {
                    st_nt(&v4[(base + offset2(s)) >> 1], *reinterpret_cast<const float4 *>(&tile[swz_p(x)]));
                } else {
                    const C lo = tile[swz(src(x))], hi = tile[swz(src(x + 1))];
                    st_nt(&v4[(base + offset2(s)) >> 1], make_float4(lo.x, lo.y, hi.x, hi.y));
                }
            }
        } else {
            C *v = reinterpret_cast<C *>(st);
#pragma unroll
            for (int s = 0; s < OPT; ++s)
                st_nt(&v[base + offset2(s)],
                      tile[PSWZ ? swz_p(uint32_t(s * NTH + tid2)) : swz(src(uint32_t(s * NTH + tid2)))]);
        }
    }
}

// Whether a tile_sweep over these tile arguments moves 16-byte amplitude
// pairs (complex64 with physical bit 0 in the tile).
inline bool tile_pairs(int dtype, const TileArgs &a)
{
    return dtype == SV_C64 && a.dep[0] == 1;
}

// Grid of a tile_sweep launch: one workgroup per tile, at most 2^22 along x
// (the thread count per dimension stays below 2^32), the rest along y.
inline dim3 tile_grid(uint64_t ntiles)
{
    const uint64_t cap = uint64_t(1) << 22;
    const uint64_t x = ntiles < 1 ? 1 : (ntiles > cap ? cap : ntiles);
    const uint64_t y = (ntiles + x - 1) / x;
    return dim3(uint32_t(x), uint32_t(y < 1 ? 1 : y));
}

inline uint64_t grid_for(uint64_t work, uint64_t per_block, uint64_t cap)
{
    uint64_t b = (work + per_block - 1) / per_block;
    if (b < 1)
        b = 1;
    return b > cap ? cap : b;
}

}  // namespace dev
}  // namespace sv
