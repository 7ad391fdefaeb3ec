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
    if (T < 1 || T > 16 || n < T || n > 63 || q > kMaxPassQubits || (phys_qmask >> n) != 0 ||
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
                       const void *d_mats, bool phases, hipStream_t s)
{
    const int T0 = pass_tile_log(dtype);
    if (nsub < 1 || (T != T0 && T != T0 + 1) || n < T)
        return hipErrorInvalidValue;
    TileArgs a{};
    std::vector<int> bits(tile_bits, tile_bits + T);
    for (int b = 0; b < T; ++b)
        a.dep[b] = uint64_t(1) << bits[b];
    a.outer = make_insert_masks(bits);
    a.ntiles = uint64_t(1) << (n - T);
    if (dtype == SV_C64)
        return T == 12 ? launch_pass_t<float, 12, kThreads>(st, a, d_subs, nsub, d_mats, phases, s)
                       : launch_pass_t<float, 13, 512>(st, a, d_subs, nsub, d_mats, phases, s);
    return T == 11 ? launch_pass_t<double, 11, kThreads>(st, a, d_subs, nsub, d_mats, phases, s)
                   : launch_pass_t<double, 12, 512>(st, a, d_subs, nsub, d_mats, phases, s);
}

}  // namespace sv
