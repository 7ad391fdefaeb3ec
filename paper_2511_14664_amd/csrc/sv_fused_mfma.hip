// Fused k-qubit blocks (k = 4..6) on the matrix cores (gfx950 MFMA).
//
// A fused block multiplies every group of 2^k amplitudes (fixed non-target
// bits) by the block's 2^k x 2^k unitary: for a tile of G groups this is the
// complex GEMM Y = U V with V the 2^k x G matrix of gathered amplitudes, the
// dense contraction that gate fusion creates (paper Sec. 2.1: fusion raises
// the linear-algebra dimension and the arithmetic intensity of a sweep).
//
// The complex product takes three real GEMMs (Gauss):
//     P1 = Ur Vr,  P2 = Ui Vi,  P3 = (Ur + Ui)(Vr + Vi),
//     Yr = P1 - P2,  Yi = P3 - P1 - P2,
// on v_mfma_f32_16x16x4f32 (complex64, FP32 accumulation) or
// v_mfma_f64_16x16x4f64 (complex128).  At k = 5 a complex64 sweep carries
// about as many matrix-core cycles as HBM cycles with four real products, so
// the fourth product is worth removing; the extra rounding is a few units in
// the last place of |U||V|.
//
// Data path per workgroup (4 waves): one tile (the k targets + the lowest
// free bits) is loaded from HBM into LDS, each wave multiplies its (group
// set, row block) pairs, results go back to LDS and out (tile_sweep).
// Operand layouts (lane l): A[i = l % 16][kk = l / 16], B[kk = l / 16][j =
// l % 16]; the accumulator layouts are given by acc_row().
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {
namespace {

using namespace dev;

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// log2 of the tile (amplitudes) for each precision and width, by measurement
// on MI355X (28 qubits, targets low / middle / high / mixed): 32 KiB complex64
// tiles give 1 KiB contiguous runs when the targets are high qubits; complex128
// keeps 16-32 KiB tiles so that four workgroups stay resident per CU.
template <typename R, int K>
struct MfmaTile {
    static constexpr int TA_LOG = 12;
};
template <int K>
struct MfmaTile<double, K> {
    static constexpr int TA_LOG = 11;
};
template <>
struct MfmaTile<double, 4> {
    static constexpr int TA_LOG = 10;
};

template <typename R>
struct Acc4;
template <>
struct Acc4<float> {
    using T = floatx4;
};
template <>
struct Acc4<double> {
    using T = doublex4;
};

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row (within the MT-row block) held by accumulator register r of lane l
// (column = lane % NT in all three shapes; FP64 interleaves the rows).
template <typename R, int MT>
__device__ __forceinline__ int acc_row(int l, int r)
{
    if constexpr (MT == 32)
        return 8 * (r / 4) + 4 * (l / 32) + (r % 4);
    else if constexpr (std::is_same<R, double>::value)
        return 4 * r + (l / 16);
    else
        return 4 * (l / 16) + r;
}

template <typename R, int K, int TA_LOG, bool PAIR>
__global__ __launch_bounds__(kThreads) void k_dense_mfma(R *__restrict__ st, const TileArgs a)
{
    using C = typename CT<R>::C;
    using AccT = typename Acc4<R>::T;
    constexpr int MT = 16, NT = 16, KT = 4;
    constexpr int D = 1 << K;
    constexpr int M = TA_LOG - K;          // group bits
    constexpr int NGS = (1 << M) / NT;     // group sets per tile
    constexpr int NMT = D / MT;            // row blocks
    constexpr int ITEMS = NGS * NMT;       // (group set, row block) pairs
    constexpr int PER_WAVE = ITEMS / 4;
    constexpr int NS = D / KT;             // k-steps
    static_assert(ITEMS % 4 == 0 && PER_WAVE >= 1, "tile shape");
    static_assert(4 % NMT == 0, "row blocks per tile must divide the 4 waves");

    __shared__ C tile[1 << TA_LOG];
    const C *U = reinterpret_cast<const C *>(a.U);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int ai = lane % MT, akk = lane / MT;   // A operand coordinates
    const int bj = lane % NT, bkk = lane / NT;   // B operand coordinates

    // Each wave keeps one row block and takes every (4 / NMT)-th group set.
    // Everything the products need besides the tile is fetched here, before
    // the tile's loads, so that its latency hides under theirs: the U
    // fragment of this lane, and the per-lane halves of the slot table.  Slot
    // lookups split as xc[r] = xc[r_lo] | xc[r_hi] (the deposit of disjoint
    // bits of r); the halves indexed by a compile-time or wave-uniform value
    // are scalar loads.
    const int mt = __builtin_amdgcn_readfirstlane(wave % NMT);
    R ur[NS], ui[NS];
    {
        const C *Urow = U + size_t(mt * MT + ai) * D + akk;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C u = Urow[s * KT];
            ur[s] = u.x;
            ui[s] = u.y;
        }
    }
    constexpr bool F64 = std::is_same<R, double>::value;
    const uint32_t xb_lane = a.xc[bkk];                            // k-step bits 0..1
    const uint32_t xo_lane = a.xc[F64 ? (lane / 16) : 4 * (lane / 16)];  // output row, lane part
    const uint32_t xo_mt = a.xc[mt * MT];                          // output row, row-block part
    uint32_t xg[PER_WAVE];
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j)
        xg[j] = group_slot(uint32_t((wave / NMT + (4 / NMT) * j) * NT + bj), a);

    tile_sweep<R, TA_LOG, PAIR>(st, a, tile, [&](C *t) {
        AccT p1[PER_WAVE], p2[PER_WAVE], p3[PER_WAVE];
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            p1[j] = AccT{};
            p2[j] = AccT{};
            p3[j] = AccT{};
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint32_t xs = uint32_t(a.xc[s * KT]) | xb_lane;
            const R us = ur[s] + ui[s];
#pragma unroll
            for (int j = 0; j < PER_WAVE; ++j) {
                const C x = t[swz(xs | xg[j])];
                p1[j] = mfma16(ur[s], x.x, p1[j]);
                p2[j] = mfma16(ui[s], x.y, p2[j]);
                p3[j] = mfma16(us, x.x + x.y, p3[j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // acc_row<R, 16>(lane, r) = lane part | register part
            const uint32_t xrow = xo_mt | xo_lane | uint32_t(a.xc[F64 ? 4 * r : r]);
#pragma unroll
            for (int j = 0; j < PER_WAVE; ++j) {
                C y;
                y.x = p1[j][r] - p2[j][r];
                y.y = p3[j][r] - p1[j][r] - p2[j][r];
                t[swz(xrow | xg[j])] = y;
            }
        }
        __syncthreads();
    });
}

template <typename R, int K, int TA_LOG = MfmaTile<R, K>::TA_LOG>
hipError_t launch_mfma(void *st, int n, const void *d_U, const int *tgt, const int *ctl, int c, hipStream_t s)
{
    if (n - c < TA_LOG)
        return hipErrorInvalidValue;
    TileArgs a = make_tile_args(n, K, tgt, ctl, c, TA_LOG, d_U);
    const dim3 grid = tile_grid(a.ntiles);
    if (tile_pairs(std::is_same<R, float>::value ? SV_C64 : SV_C128, a))
        hipLaunchKernelGGL((k_dense_mfma<R, K, TA_LOG, std::is_same<R, float>::value>), grid, dim3(kThreads), 0, s,
                           (R *)st, a);
    else
        hipLaunchKernelGGL((k_dense_mfma<R, K, TA_LOG, false>), grid, dim3(kThreads), 0, s, (R *)st, a);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// complex64 with the three-term BF16 split (k = 5, 6).  Each FP32 operand x is
// split as x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a real product
// X Y is taken as Xhi Yhi + Xhi Ylo + Xlo Yhi (the dropped Xlo Ylo term and
// the rounding of lo leave a relative error of about 2^-16 per product), on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  Operand layouts (lane l):
// A[i = l % 32][k = 8 (l / 32) + e], B[k = 8 (l / 32) + e][j = l % 32], e < 8.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8(const float *x, bf16x8 &hi, bf16x8 &lo)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h = __bf16(x[e]);
        hi[e] = h;
        lo[e] = __bf16(x[e] - float(h));
    }
}

template <int K, bool PAIR>
__global__ __launch_bounds__(kThreads) void k_dense_bf16x3(float *__restrict__ st, const TileArgs a)
{
    using C = float2;
    constexpr int TA_LOG = 12;
    constexpr int D = 1 << K;
    constexpr int TA = 1 << TA_LOG;
    constexpr int M = TA_LOG - K;
    constexpr int NGS = (1 << M) / 32;
    constexpr int NMT = D / 32;
    constexpr int ITEMS = NGS * NMT;
    constexpr int NKC = D / 16;  // k-chunks of 16
    static_assert(ITEMS == 4, "one (group set, row block) per wave");

    __shared__ C tile[TA];
    const C *U = reinterpret_cast<const C *>(a.U);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int mt = wave % NMT;
    const int gs = wave / NMT;
    const int i = lane % 32, kb = 8 * (lane / 32);
    const uint32_t xg = group_slot(uint32_t(gs * 32 + i), a);

    bf16x8 urh[NKC], url[NKC], uih[NKC], uil[NKC];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
        float re[8], im[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const C u = U[size_t(mt * 32 + i) * D + (kc * 16 + kb + e)];
            re[e] = u.x;
            im[e] = u.y;
        }
        split8(re, urh[kc], url[kc]);
        split8(im, uih[kc], uil[kc]);
    }

    tile_sweep<float, TA_LOG, PAIR>(st, a, tile, [&](C *t) {
        floatx16 accr = {}, acci = {};
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            float vr[8], vi[8], nvi[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const C x = t[swz(uint32_t(a.xc[kc * 16 + kb + e]) | xg)];
                vr[e] = x.x;
                vi[e] = x.y;
                nvi[e] = -x.y;
            }
            bf16x8 vrh, vrl, vih, vil, nvih, nvil;
            split8(vr, vrh, vrl);
            split8(vi, vih, vil);
            split8(nvi, nvih, nvil);
            accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(urh[kc], vrh, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(urh[kc], vrl, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(url[kc], vrh, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uih[kc], nvih, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uih[kc], nvil, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uil[kc], nvih, accr, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(urh[kc], vih, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(urh[kc], vil, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(url[kc], vih, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uih[kc], vrh, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uih[kc], vrl, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uil[kc], vrh, acci, 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = mt * 32 + acc_row<float, 32>(lane, r);
            C y;
            y.x = accr[r];
            y.y = acci[r];
            t[swz(uint32_t(a.xc[row]) | xg)] = y;
        }
        __syncthreads();
    });
}

template <int K>
hipError_t launch_bf16x3(void *st, int n, const void *d_U, const int *tgt, const int *ctl, int c, hipStream_t s)
{
    if (n - c < 12)
        return hipErrorInvalidValue;
    TileArgs a = make_tile_args(n, K, tgt, ctl, c, 12, d_U);
    const dim3 grid = tile_grid(a.ntiles);
    if (tile_pairs(SV_C64, a))
        hipLaunchKernelGGL((k_dense_bf16x3<K, true>), grid, dim3(kThreads), 0, s, (float *)st, a);
    else
        hipLaunchKernelGGL((k_dense_bf16x3<K, false>), grid, dim3(kThreads), 0, s, (float *)st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense_bf16x3(void *st, int n, const void *d_U, int k, const int *tgt, const int *ctl, int c,
                               hipStream_t s)
{
    switch (k) {
    case 5: return launch_bf16x3<5>(st, n, d_U, tgt, ctl, c, s);
    case 6: return launch_bf16x3<6>(st, n, d_U, tgt, ctl, c, s);
    default: return hipErrorInvalidValue;
    }
}

int mfma_tile_log(int dtype, int k)
{
    if (dtype == SV_C64) {
        switch (k) {
        case 4: return MfmaTile<float, 4>::TA_LOG;
        case 5: return MfmaTile<float, 5>::TA_LOG;
        case 6: return MfmaTile<float, 6>::TA_LOG;
        default: return -1;
        }
    }
    switch (k) {
    case 4: return MfmaTile<double, 4>::TA_LOG;
    case 5: return MfmaTile<double, 5>::TA_LOG;
    case 6: return MfmaTile<double, 6>::TA_LOG;
    default: return -1;
    }
}

hipError_t launch_dense_mfma(void *st, int n, int dtype, const void *d_U, int k, const int *tgt, const int *ctl,
                             int c, hipStream_t s)
{
    if (dtype == SV_C64) {
        switch (k) {
        case 4: return launch_mfma<float, 4>(st, n, d_U, tgt, ctl, c, s);
        case 5: return launch_mfma<float, 5>(st, n, d_U, tgt, ctl, c, s);
        case 6: return launch_mfma<float, 6>(st, n, d_U, tgt, ctl, c, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (k) {
    case 4: return launch_mfma<double, 4>(st, n, d_U, tgt, ctl, c, s);
    case 5: return launch_mfma<double, 5>(st, n, d_U, tgt, ctl, c, s);
    case 6: return launch_mfma<double, 6>(st, n, d_U, tgt, ctl, c, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sv
