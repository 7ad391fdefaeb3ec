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

__device__ __forceinline__ uint64_t insert_zeros(uint64_t g, const InsertMasks &im)
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

template <int TA_LOG>
__device__ __forceinline__ uint64_t tile_high_offset(int s, const TileArgs &a)
{
    uint64_t off = 0;
#pragma unroll
    for (int b = 8; b < TA_LOG; ++b)
        if ((s >> (b - 8)) & 1)
            off |= a.dep[b];
    return off;
}

// ---------------------------------------------------------------------------
// Software-pipelined sweep over LDS tiles.  Each workgroup walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...; the global loads of the next tile
// are issued into registers before the current tile is computed, so HBM
// traffic overlaps the arithmetic.  For complex64 with physical bit 0 inside
// the tile, amplitude pairs are moved with 16-byte accesses.
//
// compute(tile) must read the tile, __syncthreads(), write its results back
// into the same LDS slots and __syncthreads() again.
// ---------------------------------------------------------------------------
template <typename R, int TA_LOG, typename F>
__device__ __forceinline__ void tile_pipeline(R *__restrict__ st, const TileArgs &a, typename CT<R>::C *tile,
                                              F &&compute)
{
    using C = typename CT<R>::C;
    constexpr int TA = 1 << TA_LOG;
    constexpr int OPT = TA / kThreads;
    static_assert(OPT >= 2 && OPT % 2 == 0, "tile smaller than two elements per thread");
    C *v = reinterpret_cast<C *>(st);
    const int tid = threadIdx.x;
    // pair mode: x and x+1 are adjacent amplitudes (16 bytes for complex64)
    constexpr bool CAN_PAIR = std::is_same<R, float>::value;
    const bool pair = CAN_PAIR && a.dep[0] == 1;
    uint64_t off_lo = 0;
    if (pair) {
#pragma unroll
        for (int b = 0; b < 8; ++b)
            if ((tid >> b) & 1)
                off_lo |= a.dep[b + 1];
    } else {
        off_lo = tile_low_offset(tid, a);
    }
    auto hi_off = [&](int s) -> uint64_t {
        uint64_t off = 0;
        if (pair) {
#pragma unroll
            for (int b = 9; b < TA_LOG; ++b)
                if ((s >> (b - 9)) & 1)
                    off |= a.dep[b];
        } else {
#pragma unroll
            for (int b = 8; b < TA_LOG; ++b)
                if ((s >> (b - 8)) & 1)
                    off |= a.dep[b];
        }
        return off;
    };
    R bre[OPT], bim[OPT];  // separate scalars keep the prefetch in registers
    auto load = [&](uint64_t base) {
        if constexpr (CAN_PAIR) {
            if (pair) {
                const float4 *v4 = reinterpret_cast<const float4 *>(st);
#pragma unroll
                for (int s = 0; s < OPT / 2; ++s) {
                    const float4 q = v4[(base + (off_lo | hi_off(s))) >> 1];
                    bre[2 * s] = q.x;
                    bim[2 * s] = q.y;
                    bre[2 * s + 1] = q.z;
                    bim[2 * s + 1] = q.w;
                }
                return;
            }
        }
#pragma unroll
        for (int s = 0; s < OPT; ++s) {
            const C q = v[base + (off_lo | hi_off(s))];
            bre[s] = q.x;
            bim[s] = q.y;
        }
    };
    auto to_lds = [&]() {
        if constexpr (CAN_PAIR) {
            if (pair) {
#pragma unroll
                for (int s = 0; s < OPT / 2; ++s) {
                    const uint32_t x = 2u * uint32_t(s * kThreads + tid);
                    C lo, hi;
                    lo.x = bre[2 * s];
                    lo.y = bim[2 * s];
                    hi.x = bre[2 * s + 1];
                    hi.y = bim[2 * s + 1];
                    tile[swz(x)] = lo;
                    tile[swz(x + 1)] = hi;
                }
                return;
            }
        }
#pragma unroll
        for (int s = 0; s < OPT; ++s) {
            C q;
            q.x = bre[s];
            q.y = bim[s];
            tile[swz(uint32_t(s * kThreads + tid))] = q;
        }
    };
    auto store = [&](uint64_t base) {
        if constexpr (CAN_PAIR) {
            if (pair) {
                float4 *v4 = reinterpret_cast<float4 *>(st);
#pragma unroll
                for (int s = 0; s < OPT / 2; ++s) {
                    const uint32_t x = 2u * uint32_t(s * kThreads + tid);
                    const C lo = tile[swz(x)], hi = tile[swz(x + 1)];
                    v4[(base + (off_lo | hi_off(s))) >> 1] = make_float4(lo.x, lo.y, hi.x, hi.y);
                }
                return;
            }
        }
#pragma unroll
        for (int s = 0; s < OPT; ++s)
            v[base + (off_lo | hi_off(s))] = tile[swz(uint32_t(s * kThreads + tid))];
    };

    uint64_t o = blockIdx.x;
    if (o >= a.ntiles)
        return;
    uint64_t base = insert_zeros(o, a.outer) | a.cmask;
    load(base);
    for (;;) {
        to_lds();
        __syncthreads();
        const uint64_t o_next = o + gridDim.x;
        const bool more = o_next < a.ntiles;
        uint64_t base_next = 0;
        if (more) {
            base_next = insert_zeros(o_next, a.outer) | a.cmask;
            load(base_next);
        }
        compute(tile);
        store(base);
        if (!more)
            break;
        __syncthreads();  // stores have read the tile before it is refilled
        o = o_next;
        base = base_next;
    }
}

// Number of workgroups that keep every CU busy for a persistent kernel.
inline uint64_t persistent_grid(const void *kernel, uint64_t ntiles)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const uint64_t g = uint64_t(cus) * uint64_t(per_cu);
    return ntiles < g ? (ntiles > 0 ? ntiles : 1) : g;
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
