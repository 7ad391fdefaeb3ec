// LDS passes: a sequence of fused 4-qubit blocks applied to one tile per HBM
// round trip.
//
// A pass is a set Q of at most 8 qubits and the blocks of the circuit that act
// inside Q, in circuit order.  Its tile holds the amplitudes spanned by Q and
// the lowest free index bits (2^12 complex64 or 2^11 complex128 amplitudes on
// 256 threads, so that contiguous runs stay at least 128 bytes; twice that on
// 512 threads for passes of at most two (complex64) or three (complex128)
// blocks, which are bound by HBM).  Every block is applied to the tile in LDS
// before the tile goes back to HBM: the state moves once per pass instead of
// once per block, which is the same product of unitaries in the same order
// (paper Sec. 2.1: gate application as sweeps over the amplitudes; Sec. 2.2:
// gate fusion to cut the number of sweeps).
//
// Each block is a dense 16 x 16 unitary on four tile slots (smaller blocks
// are padded with identity on other tile slots by the host).  It runs as the
// complex GEMM Y = U V over the 2^(T-4) groups of the tile, with the three
// real products of the matrix-core sweep (Gauss):
//     P1 = Ur Vr, P2 = Ui Vi, P3 = (Ur + Ui)(Vr + Vi),  Yr = P1 - P2,
//     Yi = P3 - P1 - P2,
// on v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64.  The block descriptors
// are read with scalar loads; the U fragment of the next block is fetched
// while the current one is multiplied.
//
// Gates may also reach qubits outside the tile: diagonal gates with any of
// their qubits, other gates with their controls.  Those index bits are
// constant within a tile, so on each tile such a gate is a diagonal phase on
// the block's slots, or the gate itself or the identity.  A block whose gates
// reach at most four outer qubits is stored as one fused matrix per value of
// those bits and the tile picks its variant; otherwise (phase gates only) the
// phases are folded into the block's matrix as a column phase (applied before
// the block) or a row phase (after it), from a list of monomials (outer-bit
// mask, slot mask, angle) per block evaluated once per tile into LDS.
#include <cstring>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {
namespace {

using namespace dev;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R>
struct PassAcc;
template <>
struct PassAcc<float> {
    using T = floatx4;
};
template <>
struct PassAcc<double> {
    using T = doublex4;
};

__device__ __forceinline__ floatx4 mma16(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mma16(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// sin and cos of 2 pi u / 2^32 (u: fixed-point turns).  The nearest quarter
// turn k comes from the top bits, the rest x lies in [-pi/4, pi/4) and goes
// through the Taylor series of sin and cos (truncation error below
// (pi/4)^11 / 11! = 2e-9 and (pi/4)^12 / 12! = 1e-10); then the quarter-turn
// rotation.
__device__ __forceinline__ void turn_sincos(uint32_t u, float &sn, float &cs)
{
    const uint32_t k = (u + (1u << 29)) >> 30;
    const float x = float(int32_t(u - (k << 30))) * float(2.0 * M_PI / 4294967296.0);
    const float x2 = x * x;
    const float s = x * (1.0f + x2 * (-1.0f / 6 + x2 * (1.0f / 120 + x2 * (-1.0f / 5040 + x2 * (1.0f / 362880)))));
    const float c = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24 + x2 * (-1.0f / 720 + x2 * (1.0f / 40320 + x2 * (-1.0f / 3628800)))));
    sn = (k & 1) ? c : s;
    cs = (k & 1) ? s : c;
    if (k & 2)
        sn = -sn;
    if ((k + 1) & 2)
        cs = -cs;
}

// The same for 2 pi u / 2^64 in FP64: Taylor terms through x^17 (sin) and
// x^18 (cos), truncation error below (pi/4)^19 / 19! = 2e-19.
__device__ __forceinline__ void turn_sincos(uint64_t u, double &sn, double &cs)
{
    const uint64_t k = (u + (uint64_t(1) << 61)) >> 62;
    const double x = double(int64_t(u - (k << 62))) * (2.0 * M_PI / 18446744073709551616.0);
    const double x2 = x * x;
    double s = 1.0, c = 1.0;
    // Horner from the highest term: sin = x sum (-x2)^j / (2j+1)!, cos = sum (-x2)^j / (2j)!
    for (int j = 8; j >= 1; --j)
        s = 1.0 - x2 / double((2 * j) * (2 * j + 1)) * s;
    for (int j = 9; j >= 1; --j)
        c = 1.0 - x2 / double((2 * j - 1) * (2 * j)) * c;
    s *= x;
    sn = (k & 1) ? c : s;
    cs = (k & 1) ? s : c;
    if (k & 2)
        sn = -sn;
    if ((k + 1) & 2)
        cs = -cs;
}

// Integer add to an LDS word (wrapping).
__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v)
{
    atomicAdd(p, v);
}
__device__ __forceinline__ void lds_add(uint64_t *p, uint64_t v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}

// Residency target: five workgroups per CU fill the LDS with 32 KiB tiles,
// so the complex64 256-thread kernel without phase terms is held to 96
// registers (which also keeps the matrix products in VGPR form, without
// accumulator copies); the others stay at four.
template <typename R, int TA_LOG, bool PAIR, int NTH, bool PHASES>
__global__ __launch_bounds__(NTH)
__attribute__((amdgpu_waves_per_eu(NTH == kThreads && std::is_same<R, float>::value && PAIR && !PHASES ? 5 : 4)))
void k_pass(R *__restrict__ st, const TileArgs a, const PassSub *__restrict__ subs, int nsub,
            const char *__restrict__ mats)
{
    using C = typename CT<R>::C;
    using AccT = typename PassAcc<R>::T;
    constexpr int D = 16, NT = 16, KT = 4, NS = D / KT;
    constexpr int NGS = (1 << (TA_LOG - 4)) / NT;  // group sets (NMT = 1)
    constexpr int NW = NTH / 64;  // waves
    constexpr int PER_WAVE = NGS / NW;
    constexpr bool F64 = std::is_same<R, double>::value;
    static_assert(NGS % NW == 0 && PER_WAVE >= 1, "tile shape");

    __shared__ __align__(16) C tile[1 << TA_LOG];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int ai = lane % 16, akk = lane / 16;  // A operand: U[ai][4 s + akk]
    const int bj = lane % 16, bkk = lane / 16;  // B operand: V[4 s + bkk][group bj]
    const int q = lane / 16;

    // this tile's index bits outside the tile (variant selection, phase terms)
    const uint64_t tbase = insert_zeros(uint64_t(blockIdx.y) * gridDim.x + blockIdx.x, a.outer);
    // this lane's fragment of block sb's matrix: U[ai][4 s + akk], s < NS;
    // a block with variants stores one matrix per value of its selecting
    // index bits, consecutively
    auto load_u = [&](int sb, R *xr, R *xi) {
        const PassSub &d = subs[sb];
        uint32_t var = 0;
        for (uint32_t j = 0; j < d.nvar; ++j)
            var |= uint32_t((tbase >> d.vpos[j]) & 1) << j;
        const C *U = reinterpret_cast<const C *>(mats + d.u_off) + size_t(var) * (D * D) + ai * D + akk;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C u = U[s * KT];
            xr[s] = u.x;
            xi[s] = u.y;
        }
    };
    R ur[NS], ui[NS];
    load_u(0, ur, ui);  // in flight with the tile's loads

    // Per-tile phase angles of the blocks carrying phase terms, in an LDS
    // table: row pslot holds the 16 column angles (front terms) and the 16
    // row angles (back terms) of that block on this tile, in fixed-point
    // turns (exact sums wrapping mod 2 pi: 32 bits for complex64, 64 for
    // complex128).  Wave w fills the rows of term blocks w, w + NW, ...: its
    // lanes take the block's monomials e = lane, lane + 64, ... and each one
    // whose outer bits this tile has adds its turn to the row's (side, slot
    // mask) entry with an LDS atomic add (integer sums: the same in any
    // order); a subset sum over the four mask bits across lanes then gives
    // angle(c) = sum of the entries m within c.
    using TurnT = typename std::conditional<F64, uint64_t, uint32_t>::type;
    __shared__ TurnT angles[PHASES ? kMaxTermBlocks * 32 : 1];
    auto fill_angles = [&]() {
        for (int sb = 0; sb < nsub; ++sb) {
            const PassSub &d = subs[sb];
            if (d.nterm == 0 || int(d.pslot % NW) != wave)
                continue;
            const PassTerm *tm = reinterpret_cast<const PassTerm *>(mats + d.t_off);
            TurnT *row = angles + d.pslot * 32;
            if (lane < 32)
                row[lane] = 0;
            for (uint32_t e = uint32_t(lane); e < d.nterm; e += 64) {
                const PassTerm t = tm[e];
                if ((tbase & t.omask) == t.omask)
                    lds_add(&row[t.back * 16 + t.smask], TurnT(F64 ? t.turn : (t.turn >> 32)));
            }
            // this wave's LDS operations complete in order: the entries are final
            TurnT acc = lane < 32 ? row[lane] : TurnT(0);
#pragma unroll
            for (int bit = 1; bit < 16; bit <<= 1) {
                const TurnT other = __shfl_xor(acc, bit);
                if (lane & bit)
                    acc += other;
            }
            if (lane < 32)
                row[lane] = acc;
        }
    };
    // U[r][c] * exp(i (front(c) + back(r))) for this lane's fragment of a
    // block carrying phase terms (table filled for this tile)
    auto apply_phases = [&](const PassSub &d) {
        if (PHASES && d.nterm > 0) {
            const TurnT *row = angles + d.pslot * 32;
            const TurnT tb = row[16 + ai];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                R sn, cs;
                turn_sincos(TurnT(row[s * KT + akk] + tb), sn, cs);
                const R r0 = ur[s], i0 = ui[s];
                ur[s] = r0 * cs - i0 * sn;
                ui[s] = r0 * sn + i0 * cs;
            }
        }
    };

    tile_sweep<R, TA_LOG, PAIR, NTH, true, true>(st, a, tile, [&](C *t) {
        if (PHASES) {
            fill_angles();
            __syncthreads();
        }
        // phases of block sb + 1 are folded in at the end of iteration sb,
        // where no accumulator is live
        apply_phases(subs[0]);
        for (int sb = 0; sb < nsub; ++sb) {
            R nr[NS], ni[NS];
            if (sb + 1 < nsub)
                load_u(sb + 1, nr, ni);
            const PassSub &d = subs[sb];
            // LDS addresses.  The slot deposit of a group index and the XOR
            // swizzle are both linear over XOR, and the index splits into
            // disjoint lane bits (row bits from bkk or the accumulator row,
            // group bits 0..3 from bj) and wave-uniform bits (row bits from
            // the k-step or register, group bits from wave + NW j): the lane
            // parts are computed once per block, the uniform parts on the
            // scalar unit, and each access costs one XOR.
            const uint32_t x1 = d.xc[1], x2 = d.xc[2], x4 = d.xc[4], x8 = d.xc[8];
            const uint32_t xb_lane = ((bkk & 1) ? x1 : 0u) | ((bkk & 2) ? x2 : 0u);
            const uint32_t xo_lane = F64 ? (((q & 1) ? x1 : 0u) | ((q & 2) ? x2 : 0u))
                                         : (((q & 1) ? x4 : 0u) | ((q & 2) ? x8 : 0u));
            auto deposit = [&](uint32_t g) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t lo = d.tslot_m[b];
                    g = (g & lo) | ((g & ~lo) << 1);
                }
                return g;
            };
            // byte offsets into the tile (the XOR parts scale with it)
            constexpr int SH = F64 ? 4 : 3;
            const uint32_t gl = deposit(uint32_t(bj));
            const uint32_t in_lane = swz_p(xb_lane | gl) << SH, out_lane = swz_p(xo_lane | gl) << SH;
            uint32_t hj[PER_WAVE];
#pragma unroll
            for (int j = 0; j < PER_WAVE; ++j)
                hj[j] = swz_p(deposit(uint32_t(wave + NW * j) * NT)) << SH;
            char *tb = reinterpret_cast<char *>(t);
            AccT p1[PER_WAVE], p2[PER_WAVE], p3[PER_WAVE];
#pragma unroll
            for (int j = 0; j < PER_WAVE; ++j) {
                p1[j] = AccT{};
                p2[j] = AccT{};
                p3[j] = AccT{};
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint32_t ss = swz_p(d.xc[s * KT]) << SH;
                const R us = ur[s] + ui[s];
#pragma unroll
                for (int j = 0; j < PER_WAVE; ++j) {
                    const C x = *reinterpret_cast<const C *>(tb + (in_lane ^ (ss ^ hj[j])));
                    p1[j] = mma16(ur[s], x.x, p1[j]);
                    p2[j] = mma16(ui[s], x.y, p2[j]);
                    p3[j] = mma16(us, x.x + x.y, p3[j]);
                }
            }
            // Each item writes back exactly the 16 groups x 16 rows it read,
            // so no other wave touches these locations within this block:
            // only the next block (other slots) needs the barrier below.
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // accumulator row: 4 (lane / 16) + r (FP32), 4 r + lane / 16 (FP64)
                const uint32_t rr = swz_p(d.xc[F64 ? 4 * r : r]) << SH;
#pragma unroll
                for (int j = 0; j < PER_WAVE; ++j) {
                    C y;
                    y.x = p1[j][r] - p2[j][r];
                    y.y = p3[j][r] - p1[j][r] - p2[j][r];
                    *reinterpret_cast<C *>(tb + (out_lane ^ (rr ^ hj[j]))) = y;
                }
            }
            __syncthreads();
            if (sb + 1 < nsub) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    ur[s] = nr[s];
                    ui[s] = ni[s];
                }
                apply_phases(subs[sb + 1]);
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Complex64 passes with FP32-accurate split BF16 products.
//
// Each FP32 value x is split exactly into three BF16 parts, x = h + m + l
// (h = bf16(x), m = bf16(x - h), l = x - h - m, rounding to nearest: x - h
// and x - h - m are exact FP32 differences and the last has at most 8
// significant bits, so l is exact as well; |m| <= 2^-8 |x|, |l| <= 2^-16 |x|).
// A real product X Y is then the six BF16 products Xh Yh + Xh Ym + Xm Yh +
// Xh Yl + Xm Ym + Xl Yh; the three dropped ones (Xm Yl, Xl Ym, Xl Yl) are
// below 2^-23 |X||Y| together, and the BF16 products are exact in the FP32
// accumulator.  The block runs as one real contraction of the complex
// product: [Yr; Yi] = [[Ur, -Ui], [Ui, Ur]] [Vr; Vi], K = 32 real terms, on
// v_mfma_f32_16x16x32_bf16 (BF16 matrix rate, 16x that of FP32): two 16-row
// output tiles (real and imaginary rows) x six products per group set.
//
// The K index is ordered so that lane l (q = l / 16, j = l % 16) supplies
// B[8 q + 2 r + c][j] = component c of amplitude row 4 q + r of group j, and
// receives D[4 q + r][j]: each lane reads and writes the same four
// amplitudes of a group, so a block needs no barrier between group sets.
// Its A fragment A[j][8 q + 2 r + c] holds U entries of row j, column
// 4 q + r.  Products are accumulated smallest first.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// (a, b) as two BF16 values in one register, a in the low half.  The empty
// asm keeps the compiler from re-deriving either half by a separate
// conversion.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    const bf16x2_t p = {__bf16(a), __bf16(b)};
    uint32_t r = __builtin_bit_cast(uint32_t, p);
    asm("" : "+v"(r));
    return r;
}

// Exact three-part split of the pair (a, b): parts packed as by pack_bf16.
__device__ __forceinline__ void split3(float a, float b, uint32_t &h, uint32_t &m, uint32_t &l)
{
    h = pack_bf16(a, b);
    const float ra = a - __builtin_bit_cast(float, h << 16);
    const float rb = b - __builtin_bit_cast(float, h & 0xffff0000u);
    m = pack_bf16(ra, rb);
    const float sa = ra - __builtin_bit_cast(float, m << 16);
    const float sb = rb - __builtin_bit_cast(float, m & 0xffff0000u);
    l = pack_bf16(sa, sb);
}

__device__ __forceinline__ bf16x8_t as_bf16x8(const uint32_t *w)
{
    const u32x4_t v = {w[0], w[1], w[2], w[3]};
    return __builtin_bit_cast(bf16x8_t, v);
}

// acc + (Ah + Am + Al)(Bh + Bm + Bl) without the three smallest products,
// smallest first
__device__ __forceinline__ floatx4 mma_split6(const uint32_t *ah, const uint32_t *am, const uint32_t *al,
                                              const bf16x8_t &bh, const bf16x8_t &bm, const bf16x8_t &bl)
{
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al), bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(am), bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(am), bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah), bh, acc, 0, 0, 0);
    return acc;
}

// PHASES: some block carries per-tile phase terms; the blocks' matrices are
// FP32 and every workgroup applies its tile's phases and splits them.
// Otherwise the matrices come split already (pass_presplit), and the kernel
// only loads each lane's A fragments.  NTH: 256 threads (five workgroups per
// CU, for passes of several blocks) or 512 (three, for one-block passes,
// which are bound by HBM: 8 waves share a tile's loads and its one block).
template <bool PHASES, int NTH>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NTH == 256 ? (PHASES ? 4 : 5) : 1)))
void k_pass_split(float *__restrict__ st, const TileArgs a, const PassSub *__restrict__ subs, int nsub,
                  const char *__restrict__ mats)
{
    using C = float2;
    constexpr int TA_LOG = 12;
    constexpr int D = 16, NT = 16;
    constexpr int NGS = (1 << (TA_LOG - 4)) / NT;  // group sets of 16 groups
    constexpr int NW = NTH / 64;
    constexpr int PER_WAVE = NGS / NW;
    static_assert(PER_WAVE >= 1 && NGS % NW == 0, "tile shape");

    __shared__ __align__(16) C tile[1 << TA_LOG];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int q = lane / 16, j16 = lane % 16;

    const uint64_t tbase = insert_zeros(uint64_t(blockIdx.y) * gridDim.x + blockIdx.x, a.outer);
    auto variant = [&](const PassSub &d) {
        uint32_t var = 0;
        for (uint32_t v = 0; v < d.nvar; ++v)
            var |= uint32_t((tbase >> d.vpos[v]) & 1) << v;
        return var;
    };
    // PHASES: this lane's FP32 fragment of block sb, U[j16][4 q + r], r < 4
    auto load_u = [&](int sb, float *ur, float *ui) {
        const PassSub &d = subs[sb];
        const float4 *U = reinterpret_cast<const float4 *>(reinterpret_cast<const C *>(mats + d.u_off) +
                                                           size_t(variant(d)) * (D * D) + j16 * D + 4 * q);
        const float4 u0 = U[0], u1 = U[1];
        ur[0] = u0.x;
        ui[0] = u0.y;
        ur[1] = u0.z;
        ui[1] = u0.w;
        ur[2] = u1.x;
        ui[2] = u1.y;
        ur[3] = u1.z;
        ui[3] = u1.w;
    };
    // otherwise: this lane's split A fragments of block sb, in the order
    // (h, real rows), (h, imaginary rows), (m, real), (m, imag), (l, real),
    // (l, imag), four registers each
    auto load_a = [&](int sb, uint32_t *A) {
        const PassSub &d = subs[sb];
        const uint4 *P = reinterpret_cast<const uint4 *>(mats + d.u_off + size_t(variant(d)) * kPresplitBytes) + lane;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const uint4 v = P[i * 64];
            A[4 * i] = v.x;
            A[4 * i + 1] = v.y;
            A[4 * i + 2] = v.z;
            A[4 * i + 3] = v.w;
        }
    };
    float ur[4], ui[4];
    uint32_t an[PHASES ? 1 : 24];
    if constexpr (PHASES)
        load_u(0, ur, ui);  // in flight with the tile's loads
    else
        load_a(0, an);

    // per-tile phase angles, as in k_pass (fixed-point turns, 32 bits)
    __shared__ uint32_t angles[PHASES ? kMaxTermBlocks * 32 : 1];
    auto fill_angles = [&]() {
        for (int sb = 0; sb < nsub; ++sb) {
            const PassSub &d = subs[sb];
            if (d.nterm == 0 || int(d.pslot % NW) != wave)
                continue;
            const PassTerm *tm = reinterpret_cast<const PassTerm *>(mats + d.t_off);
            uint32_t *row = angles + d.pslot * 32;
            if (lane < 32)
                row[lane] = 0;
            for (uint32_t e = uint32_t(lane); e < d.nterm; e += 64) {
                const PassTerm t = tm[e];
                if ((tbase & t.omask) == t.omask)
                    lds_add(&row[t.back * 16 + t.smask], uint32_t(t.turn >> 32));
            }
            uint32_t acc = lane < 32 ? row[lane] : 0u;
#pragma unroll
            for (int bit = 1; bit < 16; bit <<= 1) {
                const uint32_t other = __shfl_xor(acc, bit);
                if (lane & bit)
                    acc += other;
            }
            if (lane < 32)
                row[lane] = acc;
        }
    };

    tile_sweep<float, TA_LOG, true, NTH, true, true>(st, a, tile, [&](C *t) {
        if (PHASES) {
            fill_angles();
            __syncthreads();
        }
        for (int sb = 0; sb < nsub; ++sb) {
            const PassSub &d = subs[sb];
            // A operands: real rows [Ur, -Ui], imaginary rows [Ui, Ur], split
            uint32_t A[24];
            if constexpr (PHASES) {
                if (d.nterm > 0) {
                    // U[r][c] exp(i (front(c) + back(r))), r = j16, c = 4 q + k
                    const uint32_t *row = angles + d.pslot * 32;
                    const uint32_t tb = row[16 + j16];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        float sn, cs;
                        turn_sincos(uint32_t(row[4 * q + k] + tb), sn, cs);
                        const float r0 = ur[k], i0 = ui[k];
                        ur[k] = r0 * cs - i0 * sn;
                        ui[k] = r0 * sn + i0 * cs;
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    split3(ur[k], -ui[k], A[k], A[8 + k], A[16 + k]);
                    split3(ui[k], ur[k], A[4 + k], A[12 + k], A[20 + k]);
                }
                if (sb + 1 < nsub)
                    load_u(sb + 1, ur, ui);
            } else {
#pragma unroll
                for (int i = 0; i < 24; ++i)
                    A[i] = an[i];
                if (sb + 1 < nsub)
                    load_a(sb + 1, an);
            }
            const uint32_t *arh = A, *aih = A + 4, *arm = A + 8, *aim = A + 12, *arl = A + 16, *ail = A + 20;
            // LDS byte offsets (XOR-linear parts, as in k_pass): lane part
            // from (q, j16), register part from the row r, wave-uniform part
            // from the group set
            const uint32_t x4 = d.xc[4], x8 = d.xc[8];
            auto deposit = [&](uint32_t g) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t lo = d.tslot_m[b];
                    g = (g & lo) | ((g & ~lo) << 1);
                }
                return g;
            };
            const uint32_t lane_off = swz_p(((q & 1) ? x4 : 0u) | ((q & 2) ? x8 : 0u) | deposit(uint32_t(j16))) << 3;
            uint32_t roff[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                roff[r] = swz_p(d.xc[r]) << 3;
            char *tb = reinterpret_cast<char *>(t);
#pragma unroll
            for (int g = 0; g < PER_WAVE; ++g) {
                const uint32_t hoff = swz_p(deposit(uint32_t(wave + NW * g) * NT)) << 3;
                float v[8];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const C x = *reinterpret_cast<const C *>(tb + (lane_off ^ (roff[r] ^ hoff)));
                    v[2 * r] = x.x;
                    v[2 * r + 1] = x.y;
                }
                uint32_t bh[4], bm[4], bl[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    split3(v[2 * r], v[2 * r + 1], bh[r], bm[r], bl[r]);
                const bf16x8_t Bh = as_bf16x8(bh), Bm = as_bf16x8(bm), Bl = as_bf16x8(bl);
                const floatx4 yr = mma_split6(arh, arm, arl, Bh, Bm, Bl);
                const floatx4 yi = mma_split6(aih, aim, ail, Bh, Bm, Bl);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    *reinterpret_cast<C *>(tb + (lane_off ^ (roff[r] ^ hoff))) = make_float2(yr[r], yi[r]);
            }
            __syncthreads();
        }
    });
}

template <typename R, int TA_LOG, int NTH>
hipError_t launch_pass_t(void *st, const TileArgs &a, const void *subs, int nsub, const void *mats, bool phases,
                         hipStream_t s)
{
    constexpr bool F32 = std::is_same<R, float>::value;
    // a pass tile always holds physical bit 0 (a pass qubit or the lowest
    // free bit), so complex64 moves 16-byte amplitude pairs
    if (F32 && a.dep[0] != 1)
        return hipErrorInvalidValue;
    const PassSub *ps = static_cast<const PassSub *>(subs);
    const char *m = static_cast<const char *>(mats);
    if (phases)
        hipLaunchKernelGGL((k_pass<R, TA_LOG, F32, NTH, true>), tile_grid(a.ntiles), dim3(NTH), 0, s, (R *)st, a, ps,
                           nsub, m);
    else
        hipLaunchKernelGGL((k_pass<R, TA_LOG, F32, NTH, false>), tile_grid(a.ntiles), dim3(NTH), 0, s, (R *)st, a, ps,
                           nsub, m);
    return hipGetLastError();
}

}  // namespace

// BF16 bits of x rounded to nearest even (x finite), as v_cvt_pk_bf16_f32.
static uint32_t bf16_rne_bits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// Host twin of split3: (a, b) -> packed parts h, m, l.
static void split3_host(float a, float b, uint32_t &h, uint32_t &m, uint32_t &l)
{
    auto part = [](float x, float &rest) {
        const uint32_t bits = bf16_rne_bits(x);
        const uint32_t w = bits << 16;
        float v;
        std::memcpy(&v, &w, 4);
        rest = x - v;  // exact
        return bits;
    };
    float ra, rb, sa, sb;
    const uint32_t ha = part(a, ra), hb = part(b, rb);
    const uint32_t ma = part(ra, sa), mb = part(rb, sb);
    h = ha | (hb << 16);
    m = ma | (mb << 16);
    l = bf16_rne_bits(sa) | (bf16_rne_bits(sb) << 16);
}

void pass_presplit(const std::complex<double> *U, void *dst)
{
    uint32_t *o = static_cast<uint32_t *>(dst);
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane / 16, j = lane % 16;
        for (int k = 0; k < 4; ++k) {
            const std::complex<double> u = U[j * 16 + 4 * q + k];
            const float re = float(u.real()), im = float(u.imag());
            uint32_t p[2][3];
            split3_host(re, -im, p[0][0], p[0][1], p[0][2]);
            split3_host(im, re, p[1][0], p[1][1], p[1][2]);
            for (int part = 0; part < 3; ++part)
                for (int rt = 0; rt < 2; ++rt)
                    o[((part * 2 + rt) * 64 + lane) * 4 + k] = p[rt][part];
        }
    }
}

int pass_tile_log(int dtype)
{
    return dtype == SV_C64 ? 12 : 11;
}

int pass_tile_log_for(int n, int dtype, int nsub)
{
    // Passes with few blocks are bound by HBM, and twice the tile (512
    // threads, 64 KiB of LDS) doubles the contiguous runs of a pass whose
    // qubits are all high; with more blocks the matrix cores bind and the
    // smaller tile, with more workgroups per CU, overlaps better.  Complex128
    // takes the larger tile up to three blocks.  Complex64 keeps the 2^12
    // tile throughout: its runs are already 128 bytes, and on MI355X the
    // 2^13 tile measured no faster for one or two blocks (whole circuits
    // 0.2-0.7 % slower with it).  Small states keep the small tile (enough
    // tiles to spread).
    const int T = pass_tile_log(dtype);
    const int few = dtype == SV_C64 ? 0 : 3;
    return (nsub <= few && n >= T + 1 + 6) ? T + 1 : T;
}

int pass_tile_bits(int n, int T, uint64_t phys_qmask, uint64_t phys_avoid, int *tile_bits)
{
    const int q = __builtin_popcountll(phys_qmask);
    if (T < 1 || T > 16 || n < T || n > 63 || q > T || (phys_qmask >> n) != 0 ||
        (phys_qmask & phys_avoid) != 0)
        return -1;
    int got = 0;
    for (int p = 0; p < n; ++p)
        if ((phys_qmask >> p) & 1)
            tile_bits[got++] = p;
    for (int p = 0; p < n && got < T; ++p)
        if (!(((phys_qmask | phys_avoid) >> p) & 1))
            tile_bits[got++] = p;
    if (got != T)
        return -1;
    std::sort(tile_bits, tile_bits + T);
    return T;
}

hipError_t launch_pass(void *st, int n, int dtype, int T, const int *tile_bits, const void *d_subs, int nsub,
                       const void *d_mats, bool phases, bool split, hipStream_t s)
{
    const int T0 = pass_tile_log(dtype);
    if (nsub < 1 || (T != T0 && T != T0 + 1) || n < T)
        return hipErrorInvalidValue;
    if (split && (dtype != SV_C64 || T != 12))
        return hipErrorInvalidValue;
    TileArgs a{};
    std::vector<int> bits(tile_bits, tile_bits + T);
    for (int b = 0; b < T; ++b)
        a.dep[b] = uint64_t(1) << bits[b];
    a.outer = make_insert_masks(bits);
    a.ntiles = uint64_t(1) << (n - T);
    if (split) {
        if (a.dep[0] != 1)
            return hipErrorInvalidValue;
        const PassSub *ps = static_cast<const PassSub *>(d_subs);
        const char *m = static_cast<const char *>(d_mats);
        // one-block passes on 512 threads: on 28-qubit tiles 0.67-0.77 ms
        // against 0.70-0.93 on 256 (most for high pass qubits), while from
        // two blocks on 256 threads are faster (2 blocks 0.775 against 0.823,
        // 4 blocks 1.11 against 1.27 ms)
        const dim3 g = tile_grid(a.ntiles);
        if (nsub == 1) {
            if (phases)
                hipLaunchKernelGGL((k_pass_split<true, 512>), g, dim3(512), 0, s, (float *)st, a, ps, nsub, m);
            else
                hipLaunchKernelGGL((k_pass_split<false, 512>), g, dim3(512), 0, s, (float *)st, a, ps, nsub, m);
        } else {
            if (phases)
                hipLaunchKernelGGL((k_pass_split<true, 256>), g, dim3(256), 0, s, (float *)st, a, ps, nsub, m);
            else
                hipLaunchKernelGGL((k_pass_split<false, 256>), g, dim3(256), 0, s, (float *)st, a, ps, nsub, m);
        }
        return hipGetLastError();
    }
    if (dtype == SV_C64)
        return T == 12 ? launch_pass_t<float, 12, kThreads>(st, a, d_subs, nsub, d_mats, phases, s)
                       : launch_pass_t<float, 13, 512>(st, a, d_subs, nsub, d_mats, phases, s);
    return T == 11 ? launch_pass_t<double, 11, kThreads>(st, a, d_subs, nsub, d_mats, phases, s)
                   : launch_pass_t<double, 12, 512>(st, a, d_subs, nsub, d_mats, phases, s);
}

}  // namespace sv
