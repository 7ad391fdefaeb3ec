// Fused k-qubit blocks (k = 4..6) on the matrix cores (gfx950 MFMA).
//
// A fused block multiplies every group of 2^k amplitudes (fixed non-target
// bits) by the block's 2^k x 2^k unitary: for a tile of G groups this is the
// complex GEMM Y = U V with V the 2^k x G matrix of gathered amplitudes, the
// dense contraction that gate fusion creates (paper Sec. 2.1: fusion raises
// the linear-algebra dimension and the arithmetic intensity of a sweep).  In
// real arithmetic Yr = Ur Vr - Ui Vi and Yi = Ur Vi + Ui Vr: four real
// MFMA products per k-step.
//
// complex64 / FP32: v_mfma_f32_32x32x2f32 (k = 5, 6) and v_mfma_f32_16x16x4f32
// (k = 4), FP32 accumulation.  complex128 / FP64: v_mfma_f64_16x16x4f64.
//
// Data path per workgroup (4 waves): the tile (targets + m lowest free bits)
// is loaded coalesced into LDS, each wave multiplies one (group set, row
// block) pair with its U fragment held in registers for the whole kernel,
// results go back to LDS and out with coalesced stores.  Operand layouts
// (lane l): A[i = l % MT][kk = l / MT], B[kk = l / NT][j = l % NT]; the
// accumulator layouts are given by acc_row().
#include "sv_device.h"
#include "sv_internal.h"

namespace sv {
namespace {

using namespace dev;

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R, int K>
struct MfmaShape;

// 16x16x4 shapes on 2048-amplitude tiles: the U fragment, the accumulators
// and the prefetched next tile all stay in registers at 4+ waves per SIMD.
// complex64
template <>
struct MfmaShape<float, 4> {
    static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4, TA_LOG = 11;
};
template <>
struct MfmaShape<float, 5> {
    static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4, TA_LOG = 11;
};
template <>
struct MfmaShape<float, 6> {
    static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4, TA_LOG = 11;
};
// complex128
template <>
struct MfmaShape<double, 4> {
    static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4, TA_LOG = 11;
};
template <>
struct MfmaShape<double, 5> {
    static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4, TA_LOG = 11;
};
template <>
struct MfmaShape<double, 6> {
    static constexpr int MT = 16, NT = 16, KT = 4, NACC = 4, TA_LOG = 11;
};

template <typename R, int NACC>
struct Acc;
template <>
struct Acc<float, 16> {
    using T = floatx16;
};
template <>
struct Acc<float, 4> {
    using T = floatx4;
};
template <>
struct Acc<double, 4> {
    using T = doublex4;
};

template <typename R, int MT, typename A>
__device__ __forceinline__ A mfma(R a, R b, A c);

template <>
__device__ __forceinline__ floatx16 mfma<float, 32, floatx16>(float a, float b, floatx16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx4 mfma<float, 16, floatx4>(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ doublex4 mfma<double, 16, doublex4>(double a, double b, doublex4 c)
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

template <typename R, int K>
__global__ __launch_bounds__(kThreads) void k_dense_mfma(R *__restrict__ st, const TileArgs a)
{
    using C = typename CT<R>::C;
    using S = MfmaShape<R, K>;
    using AccT = typename Acc<R, S::NACC>::T;
    constexpr int D = 1 << K;
    constexpr int TA = 1 << S::TA_LOG;
    constexpr int M = S::TA_LOG - K;          // group bits
    constexpr int NGS = (1 << M) / S::NT;     // group sets per tile
    constexpr int NMT = D / S::MT;            // row blocks
    constexpr int ITEMS = NGS * NMT;          // (group set, row block) pairs
    constexpr int PER_WAVE = ITEMS / 4;
    constexpr int NS = D / S::KT;             // k-steps
    static_assert(ITEMS % 4 == 0 && PER_WAVE >= 1, "tile shape");
    static_assert(4 % NMT == 0, "row blocks per tile must divide the 4 waves");

    __shared__ C tile[TA];
    const C *U = reinterpret_cast<const C *>(a.U);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int ai = lane % S::MT, akk = lane / S::MT;   // A operand coordinates
    const int bj = lane % S::NT, bkk = lane / S::NT;   // B operand coordinates

    // Each wave keeps one row block (its U fragment stays in registers) and
    // takes every (4 / NMT)-th group set.
    const int mt = wave % NMT;
    uint32_t xg[PER_WAVE];
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j)
        xg[j] = group_slot(uint32_t((wave / NMT + (4 / NMT) * j) * S::NT + bj), a);
    R ur[NS], ui[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const C u = U[size_t(mt * S::MT + ai) * D + (s * S::KT + akk)];
        ur[s] = u.x;
        ui[s] = u.y;
    }

    tile_pipeline<R, S::TA_LOG>(st, a, tile, [&](C *t) {
        AccT accr[PER_WAVE], acci[PER_WAVE];
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            accr[j] = AccT{};
            acci[j] = AccT{};
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const C x = t[swz(uint32_t(a.xc[s * S::KT + bkk]) | xg[j])];
                accr[j] = mfma<R, S::MT, AccT>(ur[s], x.x, accr[j]);
                acci[j] = mfma<R, S::MT, AccT>(ur[s], x.y, acci[j]);
                accr[j] = mfma<R, S::MT, AccT>(ui[s], -x.y, accr[j]);
                acci[j] = mfma<R, S::MT, AccT>(ui[s], x.x, acci[j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
#pragma unroll
            for (int r = 0; r < S::NACC; ++r) {
                const int row = mt * S::MT + acc_row<R, S::MT>(lane, r);
                C y;
                y.x = accr[j][r];
                y.y = acci[j][r];
                t[swz(uint32_t(a.xc[row]) | xg[j])] = y;
            }
        }
        __syncthreads();
    });
}

template <typename R, int K>
hipError_t launch_mfma(void *st, int n, const void *d_U, const int *tgt, const int *ctl, int c, hipStream_t s)
{
    using S = MfmaShape<R, K>;
    TileArgs a = make_tile_args(n, K, tgt, ctl, c, S::TA_LOG, d_U);
    static const uint64_t full = persistent_grid(reinterpret_cast<const void *>(&k_dense_mfma<R, K>), ~uint64_t(0) >> 1);
    const uint64_t grid = std::min<uint64_t>(full, a.ntiles);
    hipLaunchKernelGGL((k_dense_mfma<R, K>), dim3(grid), dim3(kThreads), 0, s, (R *)st, a);
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

template <int K>
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

    tile_pipeline<float, TA_LOG>(st, a, tile, [&](C *t) {
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
    TileArgs a = make_tile_args(n, K, tgt, ctl, c, 12, d_U);
    static const uint64_t full = persistent_grid(reinterpret_cast<const void *>(&k_dense_bf16x3<K>), ~uint64_t(0) >> 1);
    const uint64_t grid = std::min<uint64_t>(full, a.ntiles);
    hipLaunchKernelGGL((k_dense_bf16x3<K>), dim3(grid), dim3(kThreads), 0, s, (float *)st, a);
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

namespace {
}  // namespace

int mfma_tile_log(int dtype, int k)
{
    if (k < 4 || k > 6)
        return -1;
    (void)dtype;
    return MfmaShape<float, 4>::TA_LOG;
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
