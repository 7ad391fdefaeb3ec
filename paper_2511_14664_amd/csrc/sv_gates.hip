// Gate-application sweeps over the state vector (gfx950).
//
// Every kernel here is one pass over (part of) the 2^n amplitudes in HBM:
// the paper's gate application (Sec. 2.1 "State-Vector Simulation"), where a
// one-qubit gate multiplies amplitude pairs (i, i | 2^t) by its 2x2 matrix and a
// fused k-qubit block multiplies groups of 2^k amplitudes by a 2^k x 2^k matrix.
// The sweeps are bandwidth-bound, so the kernels are built around coalesced
// 16-byte loads, several independent loads in flight per thread, and an LDS
// tile for the multi-target case so that every global access is contiguous
// whatever the target bits are.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {
namespace {

using namespace dev;

constexpr int kItems = 4;


// ---------------------------------------------------------------------------
// |0...0>
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_reset(R *__restrict__ st, uint64_t nvec)
{
    // 16-byte vectors: two complex64 or one complex128 amplitude each.
    using V = typename std::conditional<std::is_same<R, float>::value, float4, double2>::type;
    V *v = reinterpret_cast<V *>(st);
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < nvec; i += stride) {
        V z{};
        if (i == 0) {
            if constexpr (std::is_same<R, float>::value)
                z.x = 1.0f;
            else
                z.x = 1.0;
        }
        st_nt(&v[i], z);  // streaming store: the state is not read back soon
    }
}

// ---------------------------------------------------------------------------
// Global access of the one-target sweeps.  NT: streaming (nontemporal) hint,
// used only when each store instruction covers whole 128-byte lines; where
// lanes write every other half-line, the two halves must meet in L2 first.
// ---------------------------------------------------------------------------
template <bool NT, typename T>
__device__ __forceinline__ T ldg(const T *p)
{
    if constexpr (NT)
        return ld_nt(p);
    else
        return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stg(T *p, T v)
{
    if constexpr (NT)
        st_nt(p, v);
    else
        *p = v;
}

// Access modes of a one-target sweep.
enum : int {
    kScalar = 0,  // one amplitude per access
    kVec = 1,     // complex64, index bit 0 free: two adjacent groups per 16-byte access
    kT0 = 2,      // complex64, target bit 0: the pair (i0, i0 + 1) is one 16-byte access
    kShfl = 3,    // complex64 target bit 1..3 (complex128: 0..2): every lane moves its own 16-byte
                  // vector, the partner vector (target bit flipped) comes from lane l ^ 2^(t-1) (2^t)
};

// ---------------------------------------------------------------------------
// Unit map of the one-target sweeps.  A unit is what one thread item touches:
// an amplitude (pair) index with the target and fixed bits removed.  Chunk w
// (one workgroup, 2^10 units) gives thread tid the units
//   u(k) = spread(w) | tid | (k >> 1) << 8 | (k & 1) << pu,   k < 4,
// where spread() leaves bit pu free.  Items 2j and 2j + 1 are 2^pu units
// apart: pu is picked so that they lie 32 or 64 KiB apart in memory, where
// the per-thread request stream, alternating between two such regions, is
// served faster by MI355X's HBM than one linear stream (an in-place 2 GiB
// sweep measured 0.68 ms against 0.72 ms).  The amplitude index of a unit is
// a bit deposit, so it is the OR of the deposits of its disjoint parts: the
// kernel deposits spread(w) | tid once and ORs the host-computed deposits of
// bits 8 and pu per item.  FULL: every unit of the chunk exists (at least
// 2^10 units), so no item is guarded.
// ---------------------------------------------------------------------------
struct UnitMap {
    uint64_t nunits;
    uint64_t pmask;  // 2^pu - 1, pu >= 9
    uint64_t d8;     // deposit of unit bit 8
    uint64_t dp;     // deposit of unit bit pu
    uint64_t fixed;  // bits set in every index (controls, fixed target)
    InsertMasks im;
};

__device__ __forceinline__ uint64_t chunk_index()
{
    return uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
}

// Unit of item 0 of thread tid in chunk w, and the unit offsets of items.
__device__ __forceinline__ uint64_t unit0(uint64_t w, int tid, uint64_t pmask)
{
    const uint64_t wb = w << 9;
    return (wb & pmask) | ((wb & ~pmask) << 1) | uint64_t(tid);
}
__device__ __forceinline__ uint64_t unit_off(int k, uint64_t pmask)
{
    return ((k & 1) ? pmask + 1 : 0) | (uint64_t(k >> 1) << 8);
}
__device__ __forceinline__ uint64_t index_off(int k, const UnitMap &m)
{
    return ((k & 1) ? m.dp : 0) | ((k >> 1) ? m.d8 : 0);
}

// ---------------------------------------------------------------------------
// One-target dense gate (controls allowed): pair (i0, i0 | 2^t) for every
// index i0 with target bit 0 and control bits 1.  Units: kVec, 16-byte
// vectors holding two such i0 (index bit 0 free); kT0, the 16-byte pair
// itself; kScalar, one i0.  Controls on index bits inside one 128-byte line
// stay out of the unit map: every amplitude of the line is read and written,
// those whose in-line controls are not all set unchanged, so the stores cover
// whole lines instead of leaving the HBM partial-line writes.
// ---------------------------------------------------------------------------
template <typename R>
struct Gate1Args {
    UnitMap m;
    uint64_t tbit;
    uint64_t lmask;  // controls inside one 128-byte line: applied per amplitude
    R u[8];          // u00, u01, u10, u11 as (re, im)
};

// Whether amplitude index i meets the in-line controls lm (all set); LM:
// the sweep has any (else the test compiles away).
template <bool LM>
__device__ __forceinline__ bool lines_on(uint64_t i, uint64_t lm)
{
    return !LM || (i & lm) == lm;
}

template <typename R, int MODE, bool NT, bool FULL, bool LM>
__global__ __launch_bounds__(kThreads) void k_gate1(R *__restrict__ st, const Gate1Args<R> a)
{
    using C = typename CT<R>::C;
    static_assert(kItems == 4 && kThreads == 256, "unit map: 8 thread bits, item bits 8 and pu");
    C m00, m01, m10, m11;
    m00.x = a.u[0], m00.y = a.u[1], m01.x = a.u[2], m01.y = a.u[3];
    m10.x = a.u[4], m10.y = a.u[5], m11.x = a.u[6], m11.y = a.u[7];
    const uint64_t w = chunk_index();
    if (w >= ((a.m.nunits + 1023) >> 10))
        return;
    const uint64_t u0 = unit0(w, int(threadIdx.x), a.m.pmask);
    constexpr bool kPairs = MODE == kVec || (MODE == kShfl && std::is_same<R, float>::value);
    const uint64_t b0 = insert_zeros(kPairs ? u0 << 1 : u0, a.m.im) | a.m.fixed;
    auto live = [&](int k) { return FULL || (u0 | unit_off(k, a.m.pmask)) < a.m.nunits; };
    if constexpr (MODE == kShfl && std::is_same<R, double>::value) {
        // complex128: lane bits 0..2 are index bits 0..2; the lane whose bit
        // t is set holds the upper partner and computes it
        C *v = reinterpret_cast<C *>(st);
        const int sx = int(a.tbit);
        const bool upper = (threadIdx.x & sx) != 0;
        C x[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (live(k))
                x[k] = ldg<NT>(&v[b0 | index_off(k, a.m)]);
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            C y;
            y.x = __shfl_xor(x[k].x, sx);
            y.y = __shfl_xor(x[k].y, sx);
            const C lo = upper ? y : x[k], hi = upper ? x[k] : y;
            const C ma = upper ? m10 : m00, mb = upper ? m11 : m01;
            const uint64_t i = b0 | index_off(k, a.m);
            stg<NT>(&v[i], lines_on<LM>(i, a.lmask) ? cmad(mb, hi, cmul(ma, lo)) : x[k]);
        }
    } else if constexpr (MODE == kVec) {
        float4 *v = reinterpret_cast<float4 *>(st);
        float4 lo[kItems], hi[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (live(k)) {
                const uint64_t i0 = b0 | index_off(k, a.m);
                lo[k] = ldg<NT>(&v[i0 >> 1]);
                hi[k] = ldg<NT>(&v[(i0 | a.tbit) >> 1]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            const uint64_t i0 = b0 | index_off(k, a.m);
            C l0 = make_float2(lo[k].x, lo[k].y), l1 = make_float2(lo[k].z, lo[k].w);
            C h0 = make_float2(hi[k].x, hi[k].y), h1 = make_float2(hi[k].z, hi[k].w);
            C a0 = cmad(m01, h0, cmul(m00, l0)), b0_ = cmad(m11, h0, cmul(m10, l0));
            C a1 = cmad(m01, h1, cmul(m00, l1)), b1 = cmad(m11, h1, cmul(m10, l1));
            if (!lines_on<LM>(i0, a.lmask))
                a0 = l0, b0_ = h0;
            if (!lines_on<LM>(i0 | 1, a.lmask))
                a1 = l1, b1 = h1;
            stg<NT>(&v[i0 >> 1], make_float4(a0.x, a0.y, a1.x, a1.y));
            stg<NT>(&v[(i0 | a.tbit) >> 1], make_float4(b0_.x, b0_.y, b1.x, b1.y));
        }
    } else if constexpr (MODE == kShfl) {
        // lane bits 0..2 are index bits 1..3; the lane whose bit t - 1 is set
        // holds the upper partners and computes them
        float4 *v = reinterpret_cast<float4 *>(st);
        const int sx = int(a.tbit >> 1);  // 2^(t-1): partner lane offset
        const bool upper = (threadIdx.x & sx) != 0;
        // (launched with full chunks only, so both lanes of a pair are live)
        float4 x[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (live(k))
                x[k] = ldg<NT>(&v[(b0 | index_off(k, a.m)) >> 1]);
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            float4 y;
            y.x = __shfl_xor(x[k].x, sx);
            y.y = __shfl_xor(x[k].y, sx);
            y.z = __shfl_xor(x[k].z, sx);
            y.w = __shfl_xor(x[k].w, sx);
            const float4 lo = upper ? y : x[k], hi = upper ? x[k] : y;
            const C l0 = make_float2(lo.x, lo.y), l1 = make_float2(lo.z, lo.w);
            const C h0 = make_float2(hi.x, hi.y), h1 = make_float2(hi.z, hi.w);
            const C ma = upper ? m10 : m00, mb = upper ? m11 : m01;
            C r0 = cmad(mb, h0, cmul(ma, l0)), r1 = cmad(mb, h1, cmul(ma, l1));
            const uint64_t i = b0 | index_off(k, a.m);
            if (!lines_on<LM>(i, a.lmask))
                r0 = make_float2(x[k].x, x[k].y);
            if (!lines_on<LM>(i | 1, a.lmask))
                r1 = make_float2(x[k].z, x[k].w);
            stg<NT>(&v[i >> 1], make_float4(r0.x, r0.y, r1.x, r1.y));
        }
    } else if constexpr (MODE == kT0) {
        float4 *v = reinterpret_cast<float4 *>(st);
        float4 x[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (live(k))
                x[k] = ldg<NT>(&v[(b0 | index_off(k, a.m)) >> 1]);
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            const C l = make_float2(x[k].x, x[k].y), h = make_float2(x[k].z, x[k].w);
            C y0 = cmad(m01, h, cmul(m00, l)), y1 = cmad(m11, h, cmul(m10, l));
            const uint64_t i = b0 | index_off(k, a.m);
            if (!lines_on<LM>(i, a.lmask))
                y0 = l, y1 = h;
            stg<NT>(&v[i >> 1], make_float4(y0.x, y0.y, y1.x, y1.y));
        }
    } else {
        C *v = reinterpret_cast<C *>(st);
        C lo[kItems], hi[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (live(k)) {
                const uint64_t i0 = b0 | index_off(k, a.m);
                lo[k] = ldg<NT>(&v[i0]);
                hi[k] = ldg<NT>(&v[i0 | a.tbit]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            const uint64_t i0 = b0 | index_off(k, a.m);
            C y0 = cmad(m01, hi[k], cmul(m00, lo[k])), y1 = cmad(m11, hi[k], cmul(m10, lo[k]));
            if (!lines_on<LM>(i0, a.lmask))
                y0 = lo[k], y1 = hi[k];
            stg<NT>(&v[i0], y0);
            stg<NT>(&v[i0 | a.tbit], y1);
        }
    }
}

// ---------------------------------------------------------------------------
// One-target diagonal gate diag(d0, d1) with controls: a[i] *= d[bit t of i]
// over the indices whose fixed bits match (controls = 1, and the target = 1
// when d0 == 1, so lines holding no such index are never read).  Fixed bits
// inside one 128-byte line are tested per amplitude, as for the dense gate.
// Units: VEC, 16-byte vectors (index bit 0 free); else single amplitudes.
// ---------------------------------------------------------------------------
template <typename R>
struct Diag1Args {
    UnitMap m;
    uint64_t tbit;
    uint64_t lmask;  // fixed bits inside one 128-byte line: applied per amplitude
    R d[4];          // d0, d1 as (re, im)
};

template <typename R, bool VEC, bool NT, bool FULL, bool LM>
__global__ __launch_bounds__(kThreads) void k_diag1(R *__restrict__ st, const Diag1Args<R> a)
{
    using C = typename CT<R>::C;
    C d0, d1;
    d0.x = a.d[0], d0.y = a.d[1], d1.x = a.d[2], d1.y = a.d[3];
    const uint64_t w = chunk_index();
    if (w >= ((a.m.nunits + 1023) >> 10))
        return;
    const uint64_t u0 = unit0(w, int(threadIdx.x), a.m.pmask);
    const uint64_t b0 = insert_zeros(VEC ? u0 << 1 : u0, a.m.im) | a.m.fixed;
    auto live = [&](int k) { return FULL || (u0 | unit_off(k, a.m.pmask)) < a.m.nunits; };
    if constexpr (VEC) {
        float4 *v = reinterpret_cast<float4 *>(st);
        float4 x[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (live(k))
                x[k] = ldg<NT>(&v[(b0 | index_off(k, a.m)) >> 1]);
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            const uint64_t i = b0 | index_off(k, a.m);
            const C x0 = make_float2(x[k].x, x[k].y), x1 = make_float2(x[k].z, x[k].w);
            C p0 = cmul((i & a.tbit) ? d1 : d0, x0), p1 = cmul(((i | 1) & a.tbit) ? d1 : d0, x1);
            if (!lines_on<LM>(i, a.lmask))
                p0 = x0;
            if (!lines_on<LM>(i | 1, a.lmask))
                p1 = x1;
            stg<NT>(&v[i >> 1], make_float4(p0.x, p0.y, p1.x, p1.y));
        }
    } else {
        C *v = reinterpret_cast<C *>(st);
        C x[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (live(k))
                x[k] = ldg<NT>(&v[b0 | index_off(k, a.m)]);
        __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (!live(k))
                continue;
            const uint64_t i = b0 | index_off(k, a.m);
            stg<NT>(&v[i], lines_on<LM>(i, a.lmask) ? cmul((i & a.tbit) ? d1 : d0, x[k]) : x[k]);
        }
    }
}

// Whether a one-target sweep's store instructions cover whole 128-byte lines:
// lanes are contiguous over the index bits below the lowest fixed or target
// position that the access vector does not absorb.
inline bool full_lines(const std::vector<int> &pos, int n, int absorbed, int amp_bytes)
{
    int p = n;
    for (int q : pos)
        if (q != absorbed)
            p = std::min(p, q);
    return (uint64_t(amp_bytes) << p) >= 128;
}

// ---------------------------------------------------------------------------
// Dense k-target gate, one group of 2^k amplitudes per thread (small states,
// where the LDS tile below does not fit).
// ---------------------------------------------------------------------------
struct GatekArgs {
    uint64_t ngroups;
    uint64_t cmask;
    InsertMasks im;
    uint64_t off[64];
    const void *U;
};

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_gatek(R *__restrict__ st, const GatekArgs a)
{
    using C = typename CT<R>::C;
    constexpr int D = 1 << K;
    C *v = reinterpret_cast<C *>(st);
    const C *U = reinterpret_cast<const C *>(a.U);
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    for (uint64_t g = uint64_t(blockIdx.x) * kThreads + threadIdx.x; g < a.ngroups; g += stride) {
        const uint64_t base = insert_zeros(g, a.im) | a.cmask;
        C x[D];
#pragma unroll
        for (int j = 0; j < D; ++j)
            x[j] = v[base + a.off[j]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            C acc = czero<C>();
#pragma unroll
            for (int c = 0; c < D; ++c)
                acc = cmad(U[r * D + c], x[c], acc);
            v[base + a.off[r]] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Dense k-target gate through an LDS tile.
//
// A tile is the 2^(k+m) amplitudes whose bits outside (targets + the m lowest
// free bits) are fixed: 2^m groups of 2^k.  Tile-local index x lists the tile
// bits in ascending physical order, so consecutive x are consecutive
// addresses in runs of at least 2^m amplitudes: loads and stores are
// coalesced whatever the targets.  In LDS, each wave owns 64 consecutive
// groups (one per lane) and a block of RB output rows; the matrix entries it
// needs are wave-uniform (scalar loads).  LDS addresses are XOR-swizzled
// (low 6 bits ^= next 6 bits) so lanes reading with a power-of-two stride hit
// distinct banks.
// ---------------------------------------------------------------------------
template <int K>
struct TileShape {
    static constexpr int TA_LOG = (K <= 5) ? 11 : 12;
    static constexpr int TA = 1 << TA_LOG;
    static constexpr int M = TA_LOG - K;  // group bits, >= 6
    static constexpr int RB = (K >= 3) ? 8 : (1 << K);
    static constexpr int OPT = TA / kThreads;
    static constexpr int PAIRS = OPT / RB;
    static constexpr int GCH = (1 << M) / 64;
};

template <typename R, int K, bool PAIR>
__global__ __launch_bounds__(kThreads) void k_tile(R *__restrict__ st, const TileArgs a)
{
    using C = typename CT<R>::C;
    using S = TileShape<K>;
    constexpr int D = 1 << K;
    __shared__ C tile[S::TA];
    const C *U = reinterpret_cast<const C *>(a.U);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    uint32_t xg[S::PAIRS];
    int rb[S::PAIRS];
#pragma unroll
    for (int j = 0; j < S::PAIRS; ++j) {
        const int p = wave + 4 * j;
        rb[j] = p / S::GCH;
        xg[j] = group_slot(uint32_t((p % S::GCH) * 64 + lane), a);
    }

    tile_sweep<R, S::TA_LOG, PAIR>(st, a, tile, [&](C *t) {
        C acc[S::PAIRS][S::RB];
#pragma unroll
        for (int j = 0; j < S::PAIRS; ++j) {
#pragma unroll
            for (int rr = 0; rr < S::RB; ++rr)
                acc[j][rr] = czero<C>();
            const C *Ur = U + size_t(rb[j]) * S::RB * D;
            for (int col = 0; col < D; ++col) {
                const C x = t[swz(uint32_t(a.xc[col]) | xg[j])];
#pragma unroll
                for (int rr = 0; rr < S::RB; ++rr)
                    acc[j][rr] = cmad(Ur[rr * D + col], x, acc[j][rr]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < S::PAIRS; ++j)
#pragma unroll
            for (int rr = 0; rr < S::RB; ++rr)
                t[swz(uint32_t(a.xc[rb[j] * S::RB + rr]) | xg[j])] = acc[j][rr];
        __syncthreads();
    });
}

// ---------------------------------------------------------------------------
// In-place exchange of index-bit fields [lo, lo+w) and [hi, hi+w).  A tile is
// the 2^(L+2w) amplitudes spanned by the L lowest index bits (L = lo bits kept
// for contiguity, none when lo = 0) and both fields; the permutation maps
// every tile onto itself, so each workgroup reads its whole tile into LDS,
// synchronises, and writes it back permuted.  Pure copies: bit-exact.
// ---------------------------------------------------------------------------
struct BitswapArgs {
    uint64_t ntiles;
    InsertMasks outer;
    uint64_t dep[12];
    int tlog;
    int L;
    int w;
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_bitswap(R *__restrict__ st, const BitswapArgs a)
{
    using C = typename CT<R>::C;
    __shared__ C tile[4096];
    C *v = reinterpret_cast<C *>(st);
    const int tid = threadIdx.x;
    const int TA = 1 << a.tlog;
    const uint32_t wm = (1u << a.w) - 1u;
    const uint32_t fmask = (wm << a.L) | (wm << (a.L + a.w));
    uint64_t off_lo = 0;
    for (int b = 0; b < 8 && b < a.tlog; ++b)
        if ((tid >> b) & 1)
            off_lo |= a.dep[b];
    const int nsteps = TA >= kThreads ? TA / kThreads : 1;
    const bool active = tid < TA;
    for (uint64_t o = blockIdx.x; o < a.ntiles; o += gridDim.x) {
        const uint64_t base = insert_zeros(o, a.outer);
        for (int s = 0; s < nsteps; ++s) {
            if (!active)
                break;
            uint64_t off = off_lo;
            for (int b = 8; b < a.tlog; ++b)
                if ((s >> (b - 8)) & 1)
                    off |= a.dep[b];
            tile[swz(uint32_t(s * kThreads + tid))] = v[base + off];
        }
        __syncthreads();
        for (int s = 0; s < nsteps; ++s) {
            if (!active)
                break;
            const uint32_t y = uint32_t(s * kThreads + tid);
            const uint32_t f1 = (y >> a.L) & wm, f2 = (y >> (a.L + a.w)) & wm;
            const uint32_t x = (y & ~fmask) | (f1 << (a.L + a.w)) | (f2 << a.L);
            uint64_t off = off_lo;
            for (int b = 8; b < a.tlog; ++b)
                if ((s >> (b - 8)) & 1)
                    off |= a.dep[b];
            v[base + off] = tile[swz(x)];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Logical-order read-out under a non-identity qubit map.
// ---------------------------------------------------------------------------
struct GatherArgs {
    uint64_t first;
    uint64_t count;
    int n;
    int qmap[SV_MAX_QUBITS];
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_gather(const R *__restrict__ st, R *__restrict__ dst,
                                                     const GatherArgs a)
{
    using C = typename CT<R>::C;
    const C *v = reinterpret_cast<const C *>(st);
    C *d = reinterpret_cast<C *>(dst);
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    for (uint64_t j = uint64_t(blockIdx.x) * kThreads + threadIdx.x; j < a.count; j += stride) {
        const uint64_t l = a.first + j;
        uint64_t p = 0;
        for (int q = 0; q < a.n; ++q)
            p |= ((l >> q) & 1) << a.qmap[q];
        d[j] = v[p];
    }
}

template <typename R>
void fill_u(R *dst, const cd *src, int count)
{
    for (int i = 0; i < count; ++i) {
        dst[2 * i] = R(src[i].real());
        dst[2 * i + 1] = R(src[i].imag());
    }
}

}  // namespace

// ===========================================================================
// Launchers
// ===========================================================================
hipError_t launch_reset(void *st, int n, int dtype, hipStream_t s)
{
    const uint64_t bytes = (uint64_t(1) << n) * (dtype == SV_C64 ? 8 : 16);
    const uint64_t nvec = bytes / 16;
    if (nvec == 0) {
        // n = 0 cannot occur (n >= 1); a 1-qubit complex64 state is 16 bytes.
        return hipErrorInvalidValue;
    }
    const uint64_t grid = grid_for(nvec, kThreads * 8, 1u << 20);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_reset<float>, dim3(grid), dim3(kThreads), 0, s, (float *)st, nvec);
    else
        hipLaunchKernelGGL(k_reset<double>, dim3(grid), dim3(kThreads), 0, s, (double *)st, nvec);
    return hipGetLastError();
}

// Unit map of a one-target sweep over the indices with the bits at pos
// removed (target and controls, or the fixed bits of a diagonal); pairs: a
// unit is a 16-byte complex64 vector (index bit 0 free).  The partner bit pu
// is the unit bit of the first amplitude bit, among those 32, 64, 16 and 128
// KiB apart in memory, that is not removed, lies above the item bits and
// inside the unit range; else bit 9 (a plain linear map).  Measured over the
// 28 targets of a 28-qubit complex64 state, back to back: 64 KiB first 0.695
// ms per sweep, 32 KiB first 0.700, linear 0.707, 16 / 128 / 256 KiB /
// 1 MiB 0.72-0.73.
static UnitMap make_unit_map(const std::vector<int> &pos, uint64_t fixed, int amp_bytes, bool pairs, uint64_t nunits)
{
    UnitMap m{};
    m.nunits = nunits;
    m.fixed = fixed;
    m.im = make_insert_masks(pos);
    const int lb = amp_bytes == 8 ? 3 : 4;
    int pu = 9;
    for (int byte_bit : {16, 15, 14, 17}) {
        const int p = byte_bit - lb;
        if (std::find(pos.begin(), pos.end(), p) != pos.end())
            continue;
        int ub = p - (pairs ? 1 : 0);
        for (int q : pos)
            if (q < p)
                --ub;
        if (ub >= 9 && (uint64_t(2) << ub) <= nunits) {
            pu = ub;
            break;
        }
    }
    m.pmask = (uint64_t(1) << pu) - 1;
    const int sh = pairs ? 1 : 0;
    m.d8 = insert_zeros(uint64_t(1) << (8 + sh), m.im);
    m.dp = insert_zeros(uint64_t(1) << (pu + sh), m.im);
    return m;
}

// Grid of a one-target sweep: one workgroup per chunk of 2^10 units.
static dim3 unit_grid(uint64_t nunits)
{
    return tile_grid((nunits + uint64_t(kThreads) * kItems - 1) / (uint64_t(kThreads) * kItems));
}

template <typename R, int MODE, bool NT, bool LM>
void launch_gate1_l(R *p, const Gate1Args<R> &a, hipStream_t s)
{
    if (a.m.nunits >= uint64_t(kThreads) * kItems)
        hipLaunchKernelGGL((k_gate1<R, MODE, NT, true, LM>), unit_grid(a.m.nunits), dim3(kThreads), 0, s, p, a);
    else
        hipLaunchKernelGGL((k_gate1<R, MODE, NT, false, LM>), unit_grid(a.m.nunits), dim3(kThreads), 0, s, p, a);
}

template <typename R, int MODE, bool NT>
void launch_gate1_t(R *p, const Gate1Args<R> &a, hipStream_t s)
{
    if (a.lmask)
        launch_gate1_l<R, MODE, NT, true>(p, a, s);
    else
        launch_gate1_l<R, MODE, NT, false>(p, a, s);
}

hipError_t launch_gate1(void *st, int n, int dtype, const cd U[4], int t, const int *ctl, int c,
                        hipStream_t s)
{
    // controls on the index bits of one 128-byte line (4 for complex64, 3 for
    // complex128) are tested per amplitude; the others shape the unit map
    const int line_bits = dtype == SV_C64 ? 4 : 3;
    std::vector<int> cpos;
    uint64_t cmask = 0, lmask = 0;
    for (int j = 0; j < c; ++j) {
        if (ctl[j] < line_bits) {
            lmask |= uint64_t(1) << ctl[j];
        } else {
            cpos.push_back(ctl[j]);
            cmask |= uint64_t(1) << ctl[j];
        }
    }
    std::vector<int> pos(cpos);
    pos.push_back(t);
    const uint64_t ngroups = uint64_t(1) << (n - 1 - int(cpos.size()));
    if (dtype == SV_C64) {
        const bool bit0_free = t != 0;
        // targets 1..3 with no control on index bits 4..8 and every chunk
        // full: each lane moves whole 16-byte vectors (whole lines per store
        // instruction, so streaming stores) and swaps halves with a partner lane
        bool mid_ctl = false;
        for (int q : cpos)
            mid_ctl = mid_ctl || q <= 8;
        const bool shfl = bit0_free && t <= 3 && !mid_ctl && ngroups >= uint64_t(kThreads) * kItems;
        const int mode = shfl ? kShfl : (bit0_free && ngroups >= 2) ? kVec : (t == 0 ? kT0 : kScalar);
        const bool nt = shfl || full_lines(pos, n, mode == kT0 ? 0 : -1, 8);
        Gate1Args<float> a{};
        if (shfl) {
            // units: all 16-byte vectors with the controls removed
            a.m = make_unit_map(cpos, cmask, 8, true, ngroups);
        } else {
            a.m = make_unit_map(pos, cmask, 8, mode == kVec, mode == kVec ? ngroups / 2 : ngroups);
        }
        a.tbit = uint64_t(1) << t;
        a.lmask = lmask;
        fill_u(a.u, U, 4);
        float *p = (float *)st;
        switch (mode * 2 + (nt ? 1 : 0)) {
        case kShfl * 2 + 1: launch_gate1_t<float, kShfl, true>(p, a, s); break;
        case kVec * 2 + 1: launch_gate1_t<float, kVec, true>(p, a, s); break;
        case kVec * 2: launch_gate1_t<float, kVec, false>(p, a, s); break;
        case kT0 * 2 + 1: launch_gate1_t<float, kT0, true>(p, a, s); break;
        case kT0 * 2: launch_gate1_t<float, kT0, false>(p, a, s); break;
        case kScalar * 2 + 1: launch_gate1_t<float, kScalar, true>(p, a, s); break;
        default: launch_gate1_t<float, kScalar, false>(p, a, s); break;
        }
    } else {
        // targets 0..2 (inside one line) with no control on index bits 3..8
        // and every chunk full: lanes move their own amplitudes, partners
        // swap through lane shuffles, stores cover whole lines
        bool mid_ctl = false;
        for (int q : cpos)
            mid_ctl = mid_ctl || q <= 8;
        const bool shfl = t < line_bits && !mid_ctl && 2 * ngroups >= uint64_t(kThreads) * kItems;
        const bool nt = shfl || full_lines(pos, n, -1, 16);
        Gate1Args<double> a{};
        if (shfl)
            a.m = make_unit_map(cpos, cmask, 16, false, 2 * ngroups);  // units: amplitudes
        else
            a.m = make_unit_map(pos, cmask, 16, false, ngroups);
        a.tbit = uint64_t(1) << t;
        a.lmask = lmask;
        fill_u(a.u, U, 4);
        if (shfl)
            launch_gate1_t<double, kShfl, true>((double *)st, a, s);
        else if (nt)
            launch_gate1_t<double, kScalar, true>((double *)st, a, s);
        else
            launch_gate1_t<double, kScalar, false>((double *)st, a, s);
    }
    return hipGetLastError();
}

template <typename R, bool VEC, bool NT, bool LM>
void launch_diag1_l(R *p, const Diag1Args<R> &a, hipStream_t s)
{
    if (a.m.nunits >= uint64_t(kThreads) * kItems)
        hipLaunchKernelGGL((k_diag1<R, VEC, NT, true, LM>), unit_grid(a.m.nunits), dim3(kThreads), 0, s, p, a);
    else
        hipLaunchKernelGGL((k_diag1<R, VEC, NT, false, LM>), unit_grid(a.m.nunits), dim3(kThreads), 0, s, p, a);
}

template <typename R, bool VEC, bool NT>
void launch_diag1_t(R *p, const Diag1Args<R> &a, hipStream_t s)
{
    if (a.lmask)
        launch_diag1_l<R, VEC, NT, true>(p, a, s);
    else
        launch_diag1_l<R, VEC, NT, false>(p, a, s);
}

hipError_t launch_diag1(void *st, int n, int dtype, cd d0, cd d1, int t, const int *ctl, int c,
                        hipStream_t s)
{
    // fixed bits (controls, and the target when d0 == 1) on the index bits of
    // one 128-byte line are tested per amplitude; the others shape the unit map
    const int line_bits = dtype == SV_C64 ? 4 : 3;
    std::vector<int> pos;
    uint64_t fixed = 0, lmask = 0;
    auto fix = [&](int q) {
        if (q < line_bits) {
            lmask |= uint64_t(1) << q;
        } else {
            pos.push_back(q);
            fixed |= uint64_t(1) << q;
        }
    };
    for (int j = 0; j < c; ++j)
        fix(ctl[j]);
    if (d0 == cd(1.0, 0.0))
        fix(t);
    const uint64_t nfree = uint64_t(1) << (n - int(pos.size()));
    const bool vec = dtype == SV_C64 && nfree >= 2;
    const bool nt = full_lines(pos, n, -1, dtype == SV_C64 ? 8 : 16);
    const cd dd[2] = {d0, d1};
    if (dtype == SV_C64) {
        Diag1Args<float> a{};
        a.m = make_unit_map(pos, fixed, 8, vec, vec ? nfree / 2 : nfree);
        a.tbit = uint64_t(1) << t;
        a.lmask = lmask;
        fill_u(a.d, dd, 2);
        float *p = (float *)st;
        if (vec && nt)
            launch_diag1_t<float, true, true>(p, a, s);
        else if (vec)
            launch_diag1_t<float, true, false>(p, a, s);
        else if (nt)
            launch_diag1_t<float, false, true>(p, a, s);
        else
            launch_diag1_t<float, false, false>(p, a, s);
    } else {
        Diag1Args<double> a{};
        a.m = make_unit_map(pos, fixed, 16, false, nfree);
        a.tbit = uint64_t(1) << t;
        a.lmask = lmask;
        fill_u(a.d, dd, 2);
        if (nt)
            launch_diag1_t<double, false, true>((double *)st, a, s);
        else
            launch_diag1_t<double, false, false>((double *)st, a, s);
    }
    return hipGetLastError();
}

namespace {

template <typename R, int K>
hipError_t launch_gatek_direct(void *st, int n, const void *d_U, const int *tgt, const int *ctl, int c,
                               hipStream_t s)
{
    GatekArgs a{};
    std::vector<int> pos(ctl, ctl + c);
    pos.insert(pos.end(), tgt, tgt + K);
    a.im = make_insert_masks(pos);
    for (int j = 0; j < c; ++j)
        a.cmask |= uint64_t(1) << ctl[j];
    for (int j = 0; j < (1 << K); ++j) {
        uint64_t off = 0;
        for (int b = 0; b < K; ++b)
            if ((j >> b) & 1)
                off |= uint64_t(1) << tgt[b];
        a.off[j] = off;
    }
    a.U = d_U;
    a.ngroups = uint64_t(1) << (n - K - c);
    const uint64_t grid = grid_for(a.ngroups, kThreads, 1u << 20);
    hipLaunchKernelGGL((k_gatek<R, K>), dim3(grid), dim3(kThreads), 0, s, (R *)st, a);
    return hipGetLastError();
}

template <typename R, int K>
hipError_t launch_tile(void *st, int n, const void *d_U, const int *tgt, const int *ctl, int c,
                       hipStream_t s)
{
    using S = TileShape<K>;
    if (n - c - K < S::M)
        return launch_gatek_direct<R, K>(st, n, d_U, tgt, ctl, c, s);
    TileArgs a = make_tile_args(n, K, tgt, ctl, c, S::TA_LOG, d_U);
    const dim3 grid = tile_grid(a.ntiles);
    if (tile_pairs(std::is_same<R, float>::value ? SV_C64 : SV_C128, a))
        hipLaunchKernelGGL((k_tile<R, K, std::is_same<R, float>::value>), grid, dim3(kThreads), 0, s, (R *)st, a);
    else
        hipLaunchKernelGGL((k_tile<R, K, false>), grid, dim3(kThreads), 0, s, (R *)st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_tile_k(void *st, int n, const void *d_U, int k, const int *tgt, const int *ctl, int c,
                         hipStream_t s)
{
    switch (k) {
    case 1: return launch_tile<R, 1>(st, n, d_U, tgt, ctl, c, s);
    case 2: return launch_tile<R, 2>(st, n, d_U, tgt, ctl, c, s);
    case 3: return launch_tile<R, 3>(st, n, d_U, tgt, ctl, c, s);
    case 4: return launch_tile<R, 4>(st, n, d_U, tgt, ctl, c, s);
    case 5: return launch_tile<R, 5>(st, n, d_U, tgt, ctl, c, s);
    case 6: return launch_tile<R, 6>(st, n, d_U, tgt, ctl, c, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int dense_path(int n, int dtype, int k, int c, int precision)
{
    if (precision == SV_PREC_BF16X3 && dtype == SV_C64 && (k == 5 || k == 6) && n - c >= 12)
        return SV_SWEEP_DENSE_BF16X3;
    const int tl = mfma_tile_log(dtype, k);
    if (tl > 0 && n - c >= tl)
        return SV_SWEEP_DENSE_MFMA;
    const int m = (k <= 5) ? 11 - k : 6;
    return (n - c - k < m) ? SV_SWEEP_GROUP : SV_SWEEP_DENSE;
}

bool pads_to_four(int n, int dtype, int c, int precision)
{
    return c + 4 < n && dense_path(n, dtype, 4, c, precision) == SV_SWEEP_DENSE_MFMA;
}

hipError_t launch_gatek(void *st, int n, int dtype, const void *d_U, int k, const int *tgt,
                        const int *ctl, int c, int precision, hipStream_t s)
{
    const int path = dense_path(n, dtype, k, c, precision);
    if (path == SV_SWEEP_DENSE_BF16X3)
        return launch_dense_bf16x3(st, n, d_U, k, tgt, ctl, c, s);
    if (path == SV_SWEEP_DENSE_MFMA)
        return launch_dense_mfma(st, n, dtype, d_U, k, tgt, ctl, c, s);
    if (dtype == SV_C64)
        return launch_tile_k<float>(st, n, d_U, k, tgt, ctl, c, s);
    return launch_tile_k<double>(st, n, d_U, k, tgt, ctl, c, s);
}

namespace {

// Bit-field exchange on the LDS tile driver: the tile is read into LDS in
// memory order and written back in memory order, each output element taken
// from the LDS slot of its source (the map swaps the tile-local bit fields
// [L, L + w) and [L + w, L + 2w), its own inverse).
template <typename R, int TLOG, bool PAIR>
__global__ __launch_bounds__(kThreads) void k_bitswap_p(R *__restrict__ st, const TileArgs a, int L, int w)
{
    using C = typename CT<R>::C;
    constexpr int TA = 1 << TLOG;
    __shared__ C tile[TA];
    const uint32_t wm = (1u << w) - 1u;
    const uint32_t fmask = (wm << L) | (wm << (L + w));
    auto src = [=](uint32_t y) {
        const uint32_t f1 = (y >> L) & wm, f2 = (y >> (L + w)) & wm;
        return (y & ~fmask) | (f1 << (L + w)) | (f2 << L);
    };
    tile_sweep<R, TLOG, PAIR>(st, a, tile, [](C *) {}, src);
}

template <typename R, int TLOG>
hipError_t launch_bitswap_p(void *st, const TileArgs &a, int L, int w, hipStream_t s)
{
    const dim3 grid = tile_grid(a.ntiles);
    if (tile_pairs(std::is_same<R, float>::value ? SV_C64 : SV_C128, a))
        hipLaunchKernelGGL((k_bitswap_p<R, TLOG, std::is_same<R, float>::value>), grid, dim3(kThreads), 0, s, (R *)st,
                           a, L, w);
    else
        hipLaunchKernelGGL((k_bitswap_p<R, TLOG, false>), grid, dim3(kThreads), 0, s, (R *)st, a, L, w);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bitswap(void *st, int n, int dtype, int lo, int hi, int w, hipStream_t s)
{
    BitswapArgs a{};
    a.w = w;
    a.L = std::min(lo, 12 - 2 * w);
    if (a.L < 0)
        a.L = 0;
    std::vector<int> tilebits;
    for (int p = 0; p < a.L; ++p)
        tilebits.push_back(p);
    for (int b = 0; b < w; ++b)
        tilebits.push_back(lo + b);
    for (int b = 0; b < w; ++b)
        tilebits.push_back(hi + b);
    a.tlog = int(tilebits.size());
    for (int b = 0; b < a.tlog; ++b)
        a.dep[b] = uint64_t(1) << tilebits[b];
    a.outer = make_insert_masks(tilebits);
    a.ntiles = uint64_t(1) << (n - a.tlog);
    if (a.tlog >= 9) {
        TileArgs t{};
        t.ntiles = a.ntiles;
        t.outer = a.outer;
        for (int b = 0; b < a.tlog; ++b)
            t.dep[b] = a.dep[b];
        switch (a.tlog * 2 + (dtype == SV_C64 ? 0 : 1)) {
        case 18: return launch_bitswap_p<float, 9>(st, t, a.L, w, s);
        case 19: return launch_bitswap_p<double, 9>(st, t, a.L, w, s);
        case 20: return launch_bitswap_p<float, 10>(st, t, a.L, w, s);
        case 21: return launch_bitswap_p<double, 10>(st, t, a.L, w, s);
        case 22: return launch_bitswap_p<float, 11>(st, t, a.L, w, s);
        case 23: return launch_bitswap_p<double, 11>(st, t, a.L, w, s);
        case 24: return launch_bitswap_p<float, 12>(st, t, a.L, w, s);
        case 25: return launch_bitswap_p<double, 12>(st, t, a.L, w, s);
        default: break;
        }
    }
    const uint64_t grid = grid_for(a.ntiles, 1, uint64_t(1) << 20);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_bitswap<float>, dim3(grid), dim3(kThreads), 0, s, (float *)st, a);
    else
        hipLaunchKernelGGL(k_bitswap<double>, dim3(grid), dim3(kThreads), 0, s, (double *)st, a);
    return hipGetLastError();
}

hipError_t launch_gather_logical(const void *st, void *dst, int n, int dtype, const int *qmap,
                                 uint64_t first, uint64_t count, hipStream_t s)
{
    GatherArgs a{};
    a.first = first;
    a.count = count;
    a.n = n;
    for (int q = 0; q < n; ++q)
        a.qmap[q] = qmap[q];
    const uint64_t grid = grid_for(count, kThreads * 4, 1u << 20);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_gather<float>, dim3(grid), dim3(kThreads), 0, s, (const float *)st, (float *)dst, a);
    else
        hipLaunchKernelGGL(k_gather<double>, dim3(grid), dim3(kThreads), 0, s, (const double *)st, (double *)dst, a);
    return hipGetLastError();
}

}  // namespace sv
