// Read-out sweeps: marginal probabilities, Pauli expectation values and
// sampling (paper Sec. 2.1 "Measurement and Sampling", shots of Sec. 2.2).
// Each is one read pass over the state; all accumulation is FP64 whatever the
// amplitude precision, with a fixed reduction order (no atomics), so results
// are reproducible run to run.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "sv_internal.h"

namespace sv {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxQ = 30;

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

struct Masks {
    uint64_t m[kMaxQ + 1];
    int n;
};

Masks make_masks(std::vector<int> pos)
{
    std::sort(pos.begin(), pos.end());
    Masks im{};
    im.n = int(pos.size());
    for (int j = 0; j < im.n; ++j)
        im.m[j] = (uint64_t(1) << pos[j]) - 1;
    return im;
}

__device__ __forceinline__ uint64_t insert_zeros(uint64_t g, const Masks &im)
{
    for (int j = 0; j < im.n; ++j) {
        const uint64_t lo = im.m[j];
        g = (g & lo) | ((g & ~lo) << 1);
    }
    return g;
}

template <typename C>
__device__ __forceinline__ double prob(C a)
{
    const double x = double(a.x), y = double(a.y);
    return x * x + y * y;
}

// Read-only sweeps read every byte once: loads carry the nontemporal hint
// (a 2 GiB read measured 0.30 ms with it, 0.33 ms without).
typedef float rd_f32x2 __attribute__((ext_vector_type(2)));
typedef float rd_f32x4 __attribute__((ext_vector_type(4)));
typedef double rd_f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldnt(const float2 *p)
{
    const rd_f32x2 q = __builtin_nontemporal_load(reinterpret_cast<const rd_f32x2 *>(p));
    return make_float2(q.x, q.y);
}
__device__ __forceinline__ float4 ldnt(const float4 *p)
{
    const rd_f32x4 q = __builtin_nontemporal_load(reinterpret_cast<const rd_f32x4 *>(p));
    return make_float4(q.x, q.y, q.z, q.w);
}
__device__ __forceinline__ double2 ldnt(const double2 *p)
{
    const rd_f64x2 q = __builtin_nontemporal_load(reinterpret_cast<const rd_f64x2 *>(p));
    return make_double2(q.x, q.y);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the 256 threads of a block; result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        sh[w] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

// ---------------------------------------------------------------------------
// Marginals.  out[x] = sum over rest index r of |a[dep(x, Q) | ins(r)]|^2.
// ---------------------------------------------------------------------------
struct MargArgs {
    uint64_t rest;        // 2^(n-m)
    uint64_t per_chunk;   // rest indices per chunk (multiple of kThreads or rest)
    uint32_t chunks;
    uint32_t nbins;
    int m;
    uint64_t qbit[kMaxQ];
    Masks rest_im;
};

__device__ __forceinline__ uint64_t dep_x(uint64_t x, const MargArgs &a)
{
    uint64_t p = 0;
    for (int b = 0; b < a.m; ++b)
        if ((x >> b) & 1)
            p |= a.qbit[b];
    return p;
}

// Block (chunk, x): one bin, a contiguous range of rest indices (coalesced).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_marg_rmajor(const R *__restrict__ st, double *__restrict__ part,
                                                          const MargArgs a)
{
    using C = typename CT<R>::C;
    __shared__ double sh[4];
    const C *v = reinterpret_cast<const C *>(st);
    const uint64_t x = blockIdx.y;
    const uint64_t xq = dep_x(x, a);
    const uint64_t r0 = uint64_t(blockIdx.x) * a.per_chunk;
    uint64_t r1 = r0 + a.per_chunk;
    if (r1 > a.rest)
        r1 = a.rest;
    double acc = 0.0;
    for (uint64_t r = r0 + threadIdx.x; r < r1; r += kThreads)
        acc += prob(v[xq | insert_zeros(r, a.rest_im)]);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0)
        part[x * a.chunks + blockIdx.x] = acc;
}

// One thread per bin, sequential over the (few) rest indices.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_marg_xmajor(const R *__restrict__ st, double *__restrict__ out,
                                                          const MargArgs a)
{
    using C = typename CT<R>::C;
    const C *v = reinterpret_cast<const C *>(st);
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    for (uint64_t x = uint64_t(blockIdx.x) * kThreads + threadIdx.x; x < a.nbins; x += stride) {
        const uint64_t xq = dep_x(x, a);
        double acc = 0.0;
        for (uint64_t r = 0; r < a.rest; ++r)
            acc += prob(v[xq | insert_zeros(r, a.rest_im)]);
        out[x] = acc;
    }
}

// out[x] = sum_c part[x * chunks + c], ascending c.
__global__ __launch_bounds__(kThreads) void k_sum_rows(const double *__restrict__ part, double *__restrict__ out,
                                                       uint64_t rows, uint32_t cols)
{
    const uint64_t x = uint64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (x >= rows)
        return;
    double acc = 0.0;
    for (uint32_t c = 0; c < cols; ++c)
        acc += part[x * cols + c];
    out[x] = acc;
}

// Wide rows: one workgroup per row, strided partial sums in a fixed order,
// then the fixed block tree.
__global__ __launch_bounds__(kThreads) void k_sum_rows_wide(const double *__restrict__ part, double *__restrict__ out,
                                                            uint32_t cols)
{
    __shared__ double sh[4];
    const double *row = part + uint64_t(blockIdx.x) * cols;
    double acc = 0.0;
    for (uint32_t c = threadIdx.x; c < cols; c += kThreads)
        acc += row[c];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0)
        out[blockIdx.x] = acc;
}

}  // namespace

// out[x] = sum over c of part[x * cols + c], x < rows, in a fixed order.
static hipError_t launch_sum_rows(const double *part, double *out, uint64_t rows, uint32_t cols, hipStream_t s)
{
    if (cols >= kThreads && rows <= (uint64_t(1) << 20)) {
        hipLaunchKernelGGL(k_sum_rows_wide, dim3(uint32_t(rows)), dim3(kThreads), 0, s, part, out, cols);
    } else {
        const uint64_t g = (rows + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_sum_rows, dim3(uint32_t(g)), dim3(kThreads), 0, s, part, out, rows, cols);
    }
    return hipGetLastError();
}

namespace {

// ---------------------------------------------------------------------------
// Z-string expectations: sum_i |a_i|^2 (-1)^popcount(i & z_t), up to kMaxZ
// strings per pass.  part[t * gridDim + block].
//
// A thread visits the indexes h0 + 256 u + threadIdx.x, u < 16, with h0 a
// multiple of 4096 that is the same across the workgroup, so the sign
// factors as (-1)^popcount(h0 & z_t) * (-1)^popcount(u & k_t) *
// (-1)^popcount(threadIdx.x & z_t), k_t = bits 8 .. 11 of z_t.  The first
// factors of all strings form one wave-uniform word per h0: lane t computes
// the parity for string t and a ballot collects them.  The second is folded
// into a Walsh transform of the thread's 16 probabilities over u, so each
// string takes one coefficient, picked by its uniform k_t, per 16
// amplitudes.  The third is applied once at the end.  Per 16 amplitudes
// and string the work is one FP64 FMA with a scalar +-1 operand (the scalar
// unit, shared by a CU's four SIMDs, otherwise bounds the sweep).
// ---------------------------------------------------------------------------
constexpr int kMaxZ = 32;
struct ExpZArgs {
    uint64_t nelem;
    int nt;
    uint64_t z[kMaxZ];
};

template <typename R, int NZ>
__global__ __launch_bounds__(kThreads) void k_expect_z(const R *__restrict__ st, double *__restrict__ part,
                                                       const ExpZArgs a)
{
    static_assert(NZ <= 64 && NZ <= kMaxZ, "one string per lane");
    using C = typename CT<R>::C;
    constexpr int LU = 4, U = 1 << LU;  // amplitudes per thread and step: index bits 8 .. 11
    static_assert(kThreads == 256, "lane and wave bits 0 .. 7");
    __shared__ double sh[4];
    const C *v = reinterpret_cast<const C *>(st);
    const int lane = threadIdx.x & 63;
    const uint64_t zl = lane < NZ ? a.z[lane] : 0;  // the string whose parity this lane reports
    double acc[NZ];
#pragma unroll
    for (int t = 0; t < NZ; ++t)
        acc[t] = 0.0;
    const uint64_t chunk = uint64_t(U) * kThreads;
    for (uint64_t h0 = uint64_t(blockIdx.x) * chunk; h0 < a.nelem; h0 += uint64_t(gridDim.x) * chunk) {
        // every load in bounds (past the end: index 0, weight 0) and all of
        // them issued before the first is used
        C x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = h0 + uint64_t(u) * kThreads + threadIdx.x;
            x[u] = ldnt(&v[i < a.nelem ? i : 0]);
        }
        __builtin_amdgcn_sched_barrier(0);
        double w[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            w[u] = h0 + uint64_t(u) * kThreads + threadIdx.x < a.nelem ? prob(x[u]) : 0.0;
        // Walsh transform over the step bits: w[k] = sum_u (-1)^popcount(u & k) p_u
#pragma unroll
        for (int b = 1; b < U; b <<= 1)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (!(u & b)) {
                    const double x = w[u], y = w[u | b];
                    w[u] = x + y;
                    w[u | b] = x - y;
                }
        // h0 has bits 0 .. 11 clear: string t's sign is (-1)^popcount(h0 & z_t)
        // (workgroup-uniform, one ballot) times coefficient k = bits 8 .. 11
        // of z_t, times the lane part applied at the end
        const uint64_t sgn = __ballot((__popcll(h0 & zl) & 1) != 0);
#pragma unroll
        for (int t = 0; t < NZ; ++t) {
            const int k = int((a.z[t] >> 8) & (U - 1));
            acc[t] = fma(((sgn >> t) & 1) ? -1.0 : 1.0, w[k], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NZ; ++t) {
        if (t < a.nt) {
            const double r = (__popc(threadIdx.x & uint32_t(a.z[t])) & 1) ? -acc[t] : acc[t];
            const double s = block_sum(r, sh);
            if (threadIdx.x == 0)
                part[uint64_t(t) * gridDim.x + blockIdx.x] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// General Pauli string, up to the i^(#Y) factor applied on the host:
// S = sum_i conj(a_{i^x}) s(i) a_i,  s(i) = (-1)^popcount(i & yz).  Pairs
// (i, i^x) with bit h (highest bit of x) of i equal to 0 are visited once.
// part[0 * grid + b] = Re, part[1 * grid + b] = Im.
// ---------------------------------------------------------------------------
struct ExpXYArgs {
    uint64_t npairs;
    uint64_t x;
    uint64_t yz;
    uint64_t hmask;  // 2^h - 1
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect_xy(const R *__restrict__ st, double *__restrict__ part,
                                                        const ExpXYArgs a)
{
    using C = typename CT<R>::C;
    __shared__ double sh[4];
    const C *v = reinterpret_cast<const C *>(st);
    double re = 0.0, im = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    for (uint64_t g = uint64_t(blockIdx.x) * kThreads + threadIdx.x; g < a.npairs; g += stride) {
        const uint64_t i = (g & a.hmask) | ((g & ~a.hmask) << 1);
        const uint64_t j = i ^ a.x;
        const C ai = v[i], aj = v[j];
        const double si = (__popcll(i & a.yz) & 1) ? -1.0 : 1.0;
        const double sj = (__popcll(j & a.yz) & 1) ? -1.0 : 1.0;
        const double air = ai.x, aii = ai.y, ajr = aj.x, aji = aj.y;
        // conj(aj) * ai * si + conj(ai) * aj * sj
        re += si * (ajr * air + aji * aii) + sj * (air * ajr + aii * aji);
        im += si * (ajr * aii - aji * air) + sj * (air * aji - aii * ajr);
    }
    const double sre = block_sum(re, sh);
    const double sim = block_sum(im, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sre;
        part[uint64_t(gridDim.x) + blockIdx.x] = sim;
    }
}

// ---------------------------------------------------------------------------
// Sampling.  Stage 1: sums of |a|^2 over blocks of 2^lbs amplitudes.
// ---------------------------------------------------------------------------
// The block is read in steps of 16 16-byte loads per thread, all issued
// before the first is used (indices past the block end: its first vector,
// weight 0).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_block_sums(const R *__restrict__ st, double *__restrict__ bs,
                                                         int lbs)
{
    constexpr bool F32 = std::is_same<R, float>::value;
    using V = typename std::conditional<F32, float4, double2>::type;  // 16 bytes
    constexpr int NL = 16;
    __shared__ double sh[4];
    const uint32_t nv = F32 ? (1u << lbs) >> 1 : (1u << lbs);  // vectors in the block (lbs >= 1)
    const V *v = reinterpret_cast<const V *>(st) + uint64_t(blockIdx.x) * nv;
    double acc = 0.0;
    for (uint32_t e0 = 0; e0 < nv; e0 += NL * kThreads) {
        V x[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const uint32_t e = e0 + uint32_t(k * kThreads) + threadIdx.x;
            x[k] = ldnt(&v[e < nv ? e : 0]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            double p;
            if constexpr (F32)
                p = prob(make_float2(x[k].x, x[k].y)) + prob(make_float2(x[k].z, x[k].w));
            else
                p = prob(x[k]);
            acc += e0 + uint32_t(k * kThreads) + threadIdx.x < nv ? p : 0.0;
        }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0)
        bs[blockIdx.x] = acc;
}

// Stage 1b (one workgroup): each shot's block and residual target from the
// block totals, on the device.  Thread c sums the totals of chunk c (nb / 1024
// consecutive blocks, or one block when nb < 1024) in order; one thread
// forms the chunks' running sums in order.  Shot s targets t = u_s * norm and
// takes the first block whose running sum (chunk start + in-chunk partial
// sum, added in the same order as the chunk total) exceeds t, with residual
// t minus the running sum before that block.  Running sums are sums of
// nonnegative terms in one fixed order, so they never decrease and the
// chunk search and the in-chunk walk agree.  A target at or past the total
// takes the last block of nonzero total with that total as residual.
constexpr int kPrepThreads = 1024;

__global__ __launch_bounds__(kPrepThreads) void k_sample_prep(const double *__restrict__ bs, uint64_t nb,
                                                              const double *__restrict__ uni, int shots,
                                                              int64_t *__restrict__ blk, double *__restrict__ tgt)
{
    __shared__ double csum[kPrepThreads];
    __shared__ double cpre[kPrepThreads + 1];
    __shared__ int64_t cnz[kPrepThreads];
    __shared__ int64_t s_last;
    const int tid = threadIdx.x;
    const uint64_t nchunk = nb < uint64_t(kPrepThreads) ? nb : uint64_t(kPrepThreads);
    const uint64_t cl = nb / nchunk;  // nb is a power of two
    if (uint64_t(tid) < nchunk) {
        double acc = 0.0;
        int64_t nz = -1;
        for (uint64_t b = uint64_t(tid) * cl; b < uint64_t(tid + 1) * cl; ++b) {
            const double x = bs[b];
            acc += x;
            if (x > 0.0)
                nz = int64_t(b);
        }
        csum[tid] = acc;
        cnz[tid] = nz;
    }
    __syncthreads();
    if (tid == 0) {
        double run = 0.0;
        int64_t last = 0;
        for (uint64_t c = 0; c < nchunk; ++c) {
            cpre[c] = run;
            run += csum[c];
            if (cnz[c] >= 0)
                last = cnz[c];
        }
        cpre[nchunk] = run;
        s_last = last;
    }
    __syncthreads();
    const double norm = cpre[nchunk];
    for (int sh = tid; sh < shots; sh += kPrepThreads) {
        const double t = uni[sh] * norm;
        uint64_t lo = 0, hi = nchunk;  // first chunk c with cpre[c + 1] > t
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (cpre[mid + 1] > t)
                hi = mid;
            else
                lo = mid + 1;
        }
        int64_t b_out = s_last;
        double t_out = bs[s_last];
        if (lo < nchunk) {
            const double start = cpre[lo];
            double part = 0.0;
            for (uint64_t b = lo * cl; b < (lo + 1) * cl; ++b) {
                const double before = part;
                part += bs[b];
                if (start + part > t) {
                    b_out = int64_t(b);
                    t_out = t - (start + before);
                    break;
                }
            }
        }
        blk[sh] = b_out;
        tgt[sh] = t_out;
    }
}

// Stage 2: one workgroup per shot walks its block in segments of 1024
// amplitudes (4 consecutive per thread) and returns the first index whose
// in-block running sum exceeds the residual target.  If rounding leaves none,
// the last index of nonzero probability in the block is returned.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_sample_search(const R *__restrict__ st,
                                                            const int64_t *__restrict__ blocks,
                                                            const double *__restrict__ targets,
                                                            int64_t *__restrict__ out, int lbs)
{
    using C = typename CT<R>::C;
    __shared__ double wsum[4];
    __shared__ int found;
    __shared__ int lastnz;
    const C *v = reinterpret_cast<const C *>(st);
    const int s = blockIdx.x;
    const uint64_t base = uint64_t(blocks[s]) << lbs;
    const double target = targets[s];
    const int bsz = 1 << lbs;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) {
        found = 0x7fffffff;
        lastnz = -1;
    }
    __syncthreads();
    double running = 0.0;
    for (int seg = 0; seg < bsz; seg += 4 * kThreads) {
        double c[4];
        double acc = 0.0;
        int mynz = -1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int off = seg + tid * 4 + e;
            double p = 0.0;
            if (off < bsz)
                p = prob(v[base + off]);
            if (p > 0.0)
                mynz = off;
            acc += p;
            c[e] = acc;
        }
        // inclusive scan of thread totals within the wave
        double inc = acc;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(inc, d, 64);
            if (lane >= d)
                inc += o;
        }
        if (lane == 63)
            wsum[w] = inc;
        __syncthreads();
        double wprefix = 0.0;
        for (int j = 0; j < w; ++j)
            wprefix += wsum[j];
        const double seg_total = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
        const double excl = running + wprefix + (inc - acc);
        int cand = 0x7fffffff;
#pragma unroll
        for (int e = 3; e >= 0; --e)
            if (excl + c[e] > target && seg + tid * 4 + e < bsz)
                cand = seg + tid * 4 + e;
        if (cand != 0x7fffffff)
            atomicMin(&found, cand);
        if (mynz >= 0)
            atomicMax(&lastnz, mynz);
        __syncthreads();
        const int f = found;
        if (f != 0x7fffffff) {
            if (tid == 0)
                out[s] = int64_t(base + uint64_t(f));
            return;
        }
        running += seg_total;
        __syncthreads();
    }
    if (tid == 0)
        out[s] = int64_t(base + uint64_t(lastnz >= 0 ? lastnz : bsz - 1));
}

// Two-stage marginal for bins above a high bit: stage 1 sums contiguous
// segments of 2^s amplitudes (16-byte loads, four independent FP64
// accumulators per thread, fixed-order tree); stage 2 maps segment sums to
// bins.  Every amplitude is read exactly once, in address order.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_segment_sums(const R *__restrict__ st, double *__restrict__ seg,
                                                           int s)
{
    __shared__ double sh[4];
    const uint64_t base = uint64_t(blockIdx.x) << s;
    const uint32_t len = 1u << s;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if constexpr (std::is_same<R, float>::value) {
        const float4 *v4 = reinterpret_cast<const float4 *>(st) + (base >> 1);
        for (uint32_t e = threadIdx.x; e < len / 2; e += 2 * kThreads) {
            const float4 q = v4[e];
            a0 += double(q.x) * q.x + double(q.y) * q.y;
            a1 += double(q.z) * q.z + double(q.w) * q.w;
            if (e + kThreads < len / 2) {
                const float4 r = v4[e + kThreads];
                a2 += double(r.x) * r.x + double(r.y) * r.y;
                a3 += double(r.z) * r.z + double(r.w) * r.w;
            }
        }
    } else {
        const double2 *v2 = reinterpret_cast<const double2 *>(st) + base;
        for (uint32_t e = threadIdx.x; e < len; e += 2 * kThreads) {
            const double2 q = v2[e];
            a0 += q.x * q.x + q.y * q.y;
            if (e + kThreads < len) {
                const double2 r = v2[e + kThreads];
                a1 += r.x * r.x + r.y * r.y;
            }
        }
    }
    const double t = block_sum((a0 + a1) + (a2 + a3), sh);
    if (threadIdx.x == 0)
        seg[blockIdx.x] = t;
}

// out[x] = sum over r of p[dep(x, Q') | ins(r, Q')] on a FP64 array of 2^nb values.
__global__ __launch_bounds__(kThreads) void k_marg_doubles(const double *__restrict__ p, double *__restrict__ out,
                                                           const MargArgs a)
{
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    for (uint64_t x = uint64_t(blockIdx.x) * kThreads + threadIdx.x; x < a.nbins; x += stride) {
        const uint64_t xq = dep_x(x, a);
        double acc = 0.0;
        for (uint64_t r = 0; r < a.rest; ++r)
            acc += p[xq | insert_zeros(r, a.rest_im)];
        out[x] = acc;
    }
}

// ---------------------------------------------------------------------------
// Marginal, stage 1 for bins with low index bits: fold each 4096-amplitude
// segment (index bits 0..11) onto its 2^lb bins (the bin bits among bits
// 0..11), summing 2^F consecutive segments per workgroup.
// red[(block << lb) | bin] = sum over the workgroup's segments and the
// segment's non-bin bits.  The probabilities of a segment go to LDS; each
// bin is summed by G consecutive lanes over interleaved rest indices and
// combined by a fixed shuffle tree, so the order of every sum is fixed.
// A thread's loads of one segment differ only in the index bits from
// fold_low_bits() up: 9..11 for c64 (a 16-byte load holds the two amplitudes
// of bit 0, the lane gives bits 1..8), 8..11 for c128 (the lane gives bits
// 0..7).  When none of those bits is a bin bit (KSUM), each
// thread sums its loads in registers first and the LDS array shrinks to the
// 2^fold_low_bits() low-bit entries (4 or 2 KiB instead of 32), which leaves room for
// more resident workgroups to keep loads in flight.
// ---------------------------------------------------------------------------
constexpr int kSegLog = 12;
struct FoldArgs {
    uint32_t binmask;   // bin bits among the segment's 12 bits
    uint32_t restmask;  // the other segment bits
    int lb;             // popcount(binmask)
    int F;              // log2 segments per workgroup
};

template <typename R>
constexpr int fold_low_bits()
{
    return std::is_same<R, float>::value ? 9 : 8;
}

// x-th value (ascending) of the integers whose set bits lie in mask.
__device__ __forceinline__ uint32_t deposit(uint32_t x, uint32_t mask)
{
    uint32_t r = 0;
    for (uint32_t m = mask; x && m; m &= m - 1, x >>= 1)
        if (x & 1)
            r |= m & (~m + 1);
    return r;
}

// Optional outputs of the same read (one read of the state for several
// read-outs): NZ > 0, the partial sums of nt <= NZ Z strings (as k_expect_z:
// a Walsh transform over the thread's 16 amplitudes of a segment, indexed by
// the index bits its loads differ in, picks one coefficient per string; the
// segment's higher bits give a workgroup-uniform sign and the lane's bits a
// sign applied once at the end), part[t * grid + block]; TOT, the total
// probability of every 2^tlog consecutive segments, tot[block * 2^(F - tlog)
// + j].
typedef double f64x16 __attribute__((ext_vector_type(16)));
struct ReadoutArgs {
    uint64_t z[kMaxZ];
    int nt;
    int tlog;
    double *zpart;
    double *tot;
};

template <typename R, bool KSUM, int NZ = 0, bool TOT = false>
__global__ __launch_bounds__(kThreads) void k_marg_fold(const R *__restrict__ st, double *__restrict__ red,
                                                        const FoldArgs a, const ReadoutArgs ra)
{
    static_assert(NZ == 0 || KSUM, "Z strings ride on the register-summed fold only");
    static_assert(NZ <= kMaxZ && NZ <= 64, "one string per lane");
    constexpr int SEG = 1 << kSegLog;
    constexpr int LOW = fold_low_bits<R>();
    constexpr int PR = KSUM ? (1 << LOW) : SEG;  // LDS entries per segment
    constexpr int MAXB = (PR + kThreads - 1) / kThreads;  // bins per thread when every thread owns whole bins
    constexpr bool F32 = std::is_same<R, float>::value;
    constexpr int NLD = F32 ? SEG / (2 * kThreads) : SEG / kThreads;  // loads per thread per segment
    __shared__ double pr[PR];
    __shared__ double sh_tot[TOT || NZ > 0 ? 4 : 1];
    const int tid = threadIdx.x;
    const uint32_t restmask = KSUM ? (a.restmask & uint32_t(PR - 1)) : a.restmask;
    const int B = 1 << a.lb;
    const int E = PR >> a.lb;  // LDS entries per bin
    const int G = B >= kThreads ? 1 : min(64, kThreads / B);
    const int gi = tid % G;
    const int bin0 = tid / G;
    const bool owner_mode = B >= kThreads;
    double acc[MAXB];
#pragma unroll
    for (int k = 0; k < MAXB; ++k)
        acc[k] = 0.0;
    // rest enumeration for the group mode: x_r = deposit(r, restmask), r = gi, gi + G, ...
    const uint32_t x_first = deposit(uint32_t(gi), restmask);
    const uint32_t x_step = deposit(uint32_t(G), restmask);
    const uint32_t d_bin0 = deposit(uint32_t(bin0), a.binmask);
    // Z strings: the lane reports string `lane`'s segment parity by ballot;
    // walsh index of a string: its bits among the loads' varying index bits
    const int lane = tid & 63;
    const uint64_t zl = (NZ > 0 && lane < NZ) ? ra.z[lane] : 0;
    double zacc[NZ > 0 ? NZ : 1];
#pragma unroll
    for (int t = 0; t < (NZ > 0 ? NZ : 1); ++t)
        zacc[t] = 0.0;
    double tsum = 0.0;
    // complex64: the next segment's loads are issued before the current
    // segment's arithmetic (a vector value: registers, not private memory)
    typedef float f32xL __attribute__((ext_vector_type(F32 ? 4 * NLD : 4)));
    f32xL qn;
    if constexpr (F32) {
        const float4 *v4 = reinterpret_cast<const float4 *>(st) + ((uint64_t(blockIdx.x) << (a.F + kSegLog)) >> 1);
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const float4 q = ldnt(&v4[tid + k * kThreads]);
            qn[4 * k] = q.x, qn[4 * k + 1] = q.y, qn[4 * k + 2] = q.z, qn[4 * k + 3] = q.w;
        }
    }
    for (uint32_t j = 0; j < (1u << a.F); ++j) {
        const uint64_t base = ((uint64_t(blockIdx.x) << a.F) | j) << kSegLog;
        // the thread's 16 probabilities, by the index bits its loads differ in
        // (c64: bit 0 and bits 9..11, as 2 k + c; c128: bits 8..11, as k); a
        // vector value, so that picking a string's coefficient by its
        // (uniform) index indexes registers rather than private memory
        f64x16 w;
        if constexpr (F32) {
            const f32xL qc = qn;
            if (j + 1 < (1u << a.F)) {
                const float4 *v4 = reinterpret_cast<const float4 *>(st) + ((base + SEG) >> 1);
#pragma unroll
                for (int k = 0; k < NLD; ++k) {
                    const float4 q = ldnt(&v4[tid + k * kThreads]);
                    qn[4 * k] = q.x, qn[4 * k + 1] = q.y, qn[4 * k + 2] = q.z, qn[4 * k + 3] = q.w;
                }
            }
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < NLD; ++k) {
                const float4 q = make_float4(qc[4 * k], qc[4 * k + 1], qc[4 * k + 2], qc[4 * k + 3]);
                const double p0 = double(q.x) * q.x + double(q.y) * q.y;
                const double p1 = double(q.z) * q.z + double(q.w) * q.w;
                if constexpr (KSUM) {
                    s0 += p0;
                    s1 += p1;
                } else {
                    const int e = 2 * (tid + k * kThreads);
                    pr[e] = p0;
                    pr[e + 1] = p1;
                }
                if constexpr (NZ > 0) {
                    w[2 * k] = p0;
                    w[2 * k + 1] = p1;
                }
            }
            if constexpr (KSUM) {
                pr[2 * tid] = s0;
                pr[2 * tid + 1] = s1;
                if constexpr (TOT)
                    tsum += s0 + s1;
            }
        } else {
            const double2 *v2 = reinterpret_cast<const double2 *>(st) + base;
            double s0 = 0.0;
#pragma unroll
            for (int k = 0; k < NLD; ++k) {
                const double2 q = ldnt(&v2[tid + k * kThreads]);
                const double p0 = q.x * q.x + q.y * q.y;
                if constexpr (KSUM)
                    s0 += p0;
                else
                    pr[tid + k * kThreads] = p0;
                if constexpr (NZ > 0)
                    w[k] = p0;
            }
            if constexpr (KSUM) {
                pr[tid] = s0;
                if constexpr (TOT)
                    tsum += s0;
            }
        }
        if constexpr (NZ > 0) {
            static_assert(NZ == 0 || NLD * (F32 ? 2 : 1) == 16, "16 probabilities per thread and segment");
            // w[k] <- sum_u (-1)^popcount(u & k) p_u
#pragma unroll
            for (int b = 1; b < 16; b <<= 1)
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (!(u & b)) {
                        const double x = w[u], y = w[u | b];
                        w[u] = x + y;
                        w[u | b] = x - y;
                    }
            const uint64_t sgn = __ballot((__popcll(base & zl) & 1) != 0);
#pragma unroll
            for (int t = 0; t < NZ; ++t) {
                const uint64_t zt = ra.z[t];
                const int k = F32 ? int((zt & 1) | (((zt >> 9) & 7) << 1)) : int((zt >> 8) & 15);
                zacc[t] = fma(((sgn >> t) & 1) ? -1.0 : 1.0, w[k], zacc[t]);
            }
        }
        if constexpr (TOT) {
            if (((j + 1) & ((1u << ra.tlog) - 1)) == 0) {
                const double tt = block_sum(tsum, sh_tot);
                if (tid == 0)
                    ra.tot[(uint64_t(blockIdx.x) << (a.F - ra.tlog)) + (j >> ra.tlog)] = tt;
                tsum = 0.0;
            }
        }
        __syncthreads();
        if (owner_mode) {
            // bins tid, tid + 256, ...; E <= 16 entries each, ascending
#pragma unroll
            for (int k = 0; k < MAXB; ++k) {
                const int bin = tid + k * kThreads;
                if (bin < B) {
                    const uint32_t db = deposit(uint32_t(bin), a.binmask);
                    double sacc = 0.0;
                    uint32_t x = 0;
                    for (int r = 0; r < E; ++r) {
                        sacc += pr[db | x];
                        x = ((x | ~restmask) + 1u) & restmask;
                    }
                    acc[k] += sacc;
                }
            }
        } else if (bin0 < B) {
            double sacc = 0.0;
            uint32_t x = x_first;
            for (int r = gi; r < E; r += G) {
                sacc += pr[d_bin0 | x];
                x = ((x | ~restmask) + x_step) & restmask;
            }
            for (int off = 1; off < G; off <<= 1)
                sacc += __shfl_xor(sacc, off, 64);
            acc[0] += sacc;
        }
        __syncthreads();
    }
    const uint64_t out0 = uint64_t(blockIdx.x) << a.lb;
    if (owner_mode) {
#pragma unroll
        for (int k = 0; k < MAXB; ++k)
            if (tid + k * kThreads < B)
                red[out0 + tid + k * kThreads] = acc[k];
    } else if (bin0 < B && gi == 0) {
        red[out0 + bin0] = acc[0];
    }
    if constexpr (NZ > 0) {
        // the lane's index bits: c64 bits 1..8, c128 bits 0..7
        const uint32_t lbits = F32 ? uint32_t(tid) << 1 : uint32_t(tid);
#pragma unroll
        for (int t = 0; t < NZ; ++t) {
            if (t < ra.nt) {
                const double r = (__popc(lbits & uint32_t(ra.z[t])) & 1) ? -zacc[t] : zacc[t];
                const double v = block_sum(r, sh_tot);
                if (tid == 0)
                    ra.zpart[uint64_t(t) * gridDim.x + blockIdx.x] = v;
            }
        }
    }
}

// Row-major bin sums over an array of doubles (stage 2 of the folded
// marginal): block (chunk, x) sums one bin over a contiguous rest range.
__global__ __launch_bounds__(kThreads) void k_marg_rmajor_d(const double *__restrict__ p, double *__restrict__ part,
                                                            const MargArgs a)
{
    __shared__ double sh[4];
    const uint64_t x = blockIdx.y;
    const uint64_t xq = dep_x(x, a);
    const uint64_t r0 = uint64_t(blockIdx.x) * a.per_chunk;
    uint64_t r1 = r0 + a.per_chunk;
    if (r1 > a.rest)
        r1 = a.rest;
    double acc = 0.0;
    for (uint64_t r = r0 + threadIdx.x; r < r1; r += kThreads)
        acc += p[xq | insert_zeros(r, a.rest_im)];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0)
        part[x * a.chunks + blockIdx.x] = acc;
}

}  // namespace

// ===========================================================================
// Launchers
// ===========================================================================
namespace {

struct MargPlan {
    bool rmajor;
    uint32_t chunks;
    uint64_t per_chunk;
};

MargPlan marg_plan(int n, int m)
{
    MargPlan p{};
    const uint64_t rest = uint64_t(1) << (n - m);
    const uint64_t nbins = uint64_t(1) << m;
    p.rmajor = rest >= 4096 && m <= 15;
    if (p.rmajor) {
        uint64_t want = std::max<uint64_t>(1, 4096 / nbins);
        uint64_t maxc = std::max<uint64_t>(1, rest / (kThreads * 16));
        uint64_t chunks = std::min(want, maxc);
        p.chunks = uint32_t(chunks);
        p.per_chunk = (rest + chunks - 1) / chunks;
    } else {
        p.chunks = 1;
        p.per_chunk = rest;
    }
    return p;
}

}  // namespace

namespace {

// Route of a marginal: direct (row- or bin-major over the state), segment
// sums (every bin bit >= 12), or a segment fold (some bin bit < 12) followed
// by row- or bin-major sums over the folded array.
struct MargRoute {
    int kind;             // 0 direct, 1 segment sums, 2 fold
    int sb;               // segment bits (kind 1)
    FoldArgs fold;        // kind 2
    int n2;               // bits of the folded array (kind 2)
    std::vector<int> q2;  // bin positions in the folded array (kind 2)
    MargPlan p2;          // plan over the folded array (kind 2)
    uint64_t red;         // doubles of the folded / segment array
    uint64_t scratch;     // doubles of scratch in all
};

constexpr uint64_t kMaxFolded = uint64_t(1) << 24;  // doubles

// The fold route with 2^F segments per workgroup (the caller checks that
// bits 12 .. 12 + F - 1 hold no bin and that n >= 14).
MargRoute fold_route(int n, int m, const int *phys_q, int F)
{
    MargRoute r{};
    uint32_t binmask = 0;
    for (int b = 0; b < m; ++b)
        if (phys_q[b] < kSegLog)
            binmask |= 1u << phys_q[b];
    const int lb = __builtin_popcount(binmask);
    const int n2 = n - kSegLog - F + lb;
    r.kind = 2;
    r.fold.binmask = binmask;
    r.fold.restmask = ((1u << kSegLog) - 1u) & ~binmask;
    r.fold.lb = lb;
    r.fold.F = F;
    r.n2 = n2;
    r.red = uint64_t(1) << n2;
    r.q2.resize(size_t(m));
    for (int b = 0; b < m; ++b) {
        const int q = phys_q[b];
        r.q2[size_t(b)] = q < kSegLog ? __builtin_popcount(binmask & ((1u << q) - 1u)) : lb + q - kSegLog - F;
    }
    r.p2 = marg_plan(n2, m);
    if (!r.p2.rmajor && m <= 15) {
        // few rest entries per bin: still one workgroup per bin (a thread per
        // bin would leave the GPU nearly empty for up to 2^15 bins)
        r.p2.rmajor = true;
        r.p2.chunks = 1;
        r.p2.per_chunk = uint64_t(1) << (n2 - m);
    }
    r.scratch = r.red + (r.p2.rmajor ? (uint64_t(1) << m) * r.p2.chunks : 0);
    return r;
}

MargRoute marg_route(int n, int m, const int *phys_q)
{
    MargRoute r{};
    int b0 = n;
    uint32_t binmask = 0;
    uint64_t hibins = 0;
    for (int b = 0; b < m; ++b) {
        b0 = std::min(b0, phys_q[b]);
        if (phys_q[b] < kSegLog)
            binmask |= 1u << phys_q[b];
        else
            hibins |= uint64_t(1) << phys_q[b];
    }
    if (n >= kSegLog && b0 >= kSegLog) {
        r.kind = 1;
        r.sb = std::min(b0, 16);
        r.red = uint64_t(1) << (n - r.sb);
        r.scratch = r.red;
        return r;
    }
    const int lb = __builtin_popcount(binmask);
    if (n >= kSegLog + 2 && lb <= 10) {
        // fold F more segment bits per workgroup (non-bin bits just above 12)
        // until the folded array is at most kMaxFolded doubles
        int F = 0;
        while (F < n - kSegLog - 1 && !((hibins >> (kSegLog + F)) & 1) &&
               (uint64_t(1) << (n - kSegLog - F + lb)) > kMaxFolded)
            ++F;
        if ((uint64_t(1) << (n - kSegLog - F + lb)) <= 4 * kMaxFolded)
            return fold_route(n, m, phys_q, F);
    }
    const MargPlan p = marg_plan(n, m);
    r.kind = 0;
    r.scratch = p.rmajor ? (uint64_t(1) << m) * p.chunks : 1;
    return r;
}

}  // namespace

uint64_t marginal_scratch_doubles(int n, int m, const int *phys_q)
{
    return std::max<uint64_t>(1, marg_route(n, m, phys_q).scratch);
}

hipError_t launch_marginal(const void *st, int n, int dtype, const int *phys_q, int m, double *d_scratch,
                           double *d_out, hipStream_t s)
{
    if (m < 0 || m > kMaxQ || m > n)
        return hipErrorInvalidValue;
    const MargRoute route = marg_route(n, m, phys_q);
    if (route.kind == 1) {
        const int sb = route.sb;
        const uint64_t nseg = uint64_t(1) << (n - sb);
        if (dtype == SV_C64)
            hipLaunchKernelGGL(k_segment_sums<float>, dim3(uint32_t(nseg)), dim3(kThreads), 0, s, (const float *)st,
                               d_scratch, sb);
        else
            hipLaunchKernelGGL(k_segment_sums<double>, dim3(uint32_t(nseg)), dim3(kThreads), 0, s, (const double *)st,
                               d_scratch, sb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        MargArgs a2{};
        a2.m = m;
        a2.rest = uint64_t(1) << (n - sb - m);
        a2.nbins = uint32_t(1u << m);
        std::vector<int> q2(phys_q, phys_q + m);
        for (int b = 0; b < m; ++b) {
            q2[b] -= sb;
            a2.qbit[b] = uint64_t(1) << q2[b];
        }
        a2.rest_im = make_masks(q2);
        const uint64_t g = std::min<uint64_t>((uint64_t(a2.nbins) + kThreads - 1) / kThreads, 1u << 20);
        hipLaunchKernelGGL(k_marg_doubles, dim3(g), dim3(kThreads), 0, s, d_scratch, d_out, a2);
        return hipGetLastError();
    }
    if (route.kind == 2) {
        const uint64_t nblk = uint64_t(1) << (n - kSegLog - route.fold.F);
        if (dtype == SV_C64) {
            if ((route.fold.binmask >> fold_low_bits<float>()) == 0)
                hipLaunchKernelGGL((k_marg_fold<float, true>), dim3(uint32_t(nblk)), dim3(kThreads), 0, s,
                                   (const float *)st, d_scratch, route.fold, ReadoutArgs{});
            else
                hipLaunchKernelGGL((k_marg_fold<float, false>), dim3(uint32_t(nblk)), dim3(kThreads), 0, s,
                                   (const float *)st, d_scratch, route.fold, ReadoutArgs{});
        } else {
            if ((route.fold.binmask >> fold_low_bits<double>()) == 0)
                hipLaunchKernelGGL((k_marg_fold<double, true>), dim3(uint32_t(nblk)), dim3(kThreads), 0, s,
                                   (const double *)st, d_scratch, route.fold, ReadoutArgs{});
            else
                hipLaunchKernelGGL((k_marg_fold<double, false>), dim3(uint32_t(nblk)), dim3(kThreads), 0, s,
                                   (const double *)st, d_scratch, route.fold, ReadoutArgs{});
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        MargArgs a2{};
        a2.m = m;
        a2.rest = uint64_t(1) << (route.n2 - m);
        a2.nbins = uint32_t(1u << m);
        for (int b = 0; b < m; ++b)
            a2.qbit[b] = uint64_t(1) << route.q2[size_t(b)];
        a2.rest_im = make_masks(route.q2);
        a2.chunks = route.p2.chunks;
        a2.per_chunk = route.p2.per_chunk;
        const double *red = d_scratch;
        if (route.p2.rmajor) {
            double *part = d_scratch + route.red;
            hipLaunchKernelGGL(k_marg_rmajor_d, dim3(a2.chunks, a2.nbins), dim3(kThreads), 0, s, red, part, a2);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
            return launch_sum_rows(part, d_out, uint64_t(a2.nbins), a2.chunks, s);
        } else {
            const uint64_t g = std::min<uint64_t>((uint64_t(a2.nbins) + kThreads - 1) / kThreads, 1u << 20);
            hipLaunchKernelGGL(k_marg_doubles, dim3(g), dim3(kThreads), 0, s, red, d_out, a2);
        }
        return hipGetLastError();
    }
    MargArgs a{};
    a.m = m;
    a.rest = uint64_t(1) << (n - m);
    a.nbins = uint32_t(1u << m);
    for (int b = 0; b < m; ++b)
        a.qbit[b] = uint64_t(1) << phys_q[b];
    a.rest_im = make_masks(std::vector<int>(phys_q, phys_q + m));
    MargPlan p = marg_plan(n, m);
    a.chunks = p.chunks;
    a.per_chunk = p.per_chunk;
    if (p.rmajor) {
        dim3 grid(p.chunks, a.nbins);
        if (dtype == SV_C64)
            hipLaunchKernelGGL(k_marg_rmajor<float>, grid, dim3(kThreads), 0, s, (const float *)st, d_scratch, a);
        else
            hipLaunchKernelGGL(k_marg_rmajor<double>, grid, dim3(kThreads), 0, s, (const double *)st, d_scratch, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        return launch_sum_rows(d_scratch, d_out, uint64_t(a.nbins), p.chunks, s);
    } else {
        const uint64_t g = std::min<uint64_t>((uint64_t(a.nbins) + kThreads - 1) / kThreads, 1u << 20);
        if (dtype == SV_C64)
            hipLaunchKernelGGL(k_marg_xmajor<float>, dim3(g), dim3(kThreads), 0, s, (const float *)st, d_out, a);
        else
            hipLaunchKernelGGL(k_marg_xmajor<double>, dim3(g), dim3(kThreads), 0, s, (const double *)st, d_out, a);
    }
    return hipGetLastError();
}

namespace {
constexpr uint32_t kExpGrid = 4096;
uint32_t exp_grid(int n)
{
    const uint64_t need = ((uint64_t(1) << n) + kThreads * 16 - 1) / (kThreads * 16);
    return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(kExpGrid, need)));
}
}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free expectation entry point
// (sv_expect_pauli_noalloc): the per-workgroup partial sums of one batch of
// strings, then two result doubles per string.  Every device the library
// runs on holds its own copy until the process ends.  In host code the
// name `scratch` is a host-side stand-in, not a device address: the address
// comes from hipGetSymbolAddress, looked up once per device with that device
// current, and only that address is handed to kernels and copies.
// ---------------------------------------------------------------------------
constexpr uint64_t kNoAllocDoubles = uint64_t(kMaxZ) * kExpGrid + 2 * uint64_t(SV_NOALLOC_MAX_TERMS);
static __device__ __align__(256) double scratch[kNoAllocDoubles];

int noalloc_scratch(int device, double **ptr, uint64_t *doubles)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d outside 0..%d", device, kMaxDevices - 1);
        return SV_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (addr[device] == nullptr) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess || cur != device) {
            set_error("scratch lookup needs device %d current (current %d)", device, cur);
            return SV_EDEVICE;
        }
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return SV_EDEVICE;
        }
        addr[device] = static_cast<double *>(p);
    }
    *ptr = addr[device];
    *doubles = kNoAllocDoubles;
    return SV_OK;
}

uint64_t expect_scratch_doubles(int n)
{
    (void)n;
    return uint64_t(kMaxZ) * kExpGrid;
}

int expect_z_batch()
{
    return kMaxZ;
}

hipError_t launch_expect_z(const void *st, int n, int dtype, const uint64_t *zmasks, int nt, double *d_scratch,
                           double *d_out, hipStream_t s)
{
    if (nt < 1 || nt > kMaxZ)
        return hipErrorInvalidValue;
    ExpZArgs a{};
    a.nelem = uint64_t(1) << n;
    a.nt = nt;
    for (int t = 0; t < nt; ++t)
        a.z[t] = zmasks[t];
    const uint32_t grid = exp_grid(n);
    const dim3 g(grid), b(kThreads);
    if (dtype == SV_C64) {
        const float *p = (const float *)st;
        if (nt <= 8)
            hipLaunchKernelGGL((k_expect_z<float, 8>), g, b, 0, s, p, d_scratch, a);
        else if (nt <= 16)
            hipLaunchKernelGGL((k_expect_z<float, 16>), g, b, 0, s, p, d_scratch, a);
        else
            hipLaunchKernelGGL((k_expect_z<float, 32>), g, b, 0, s, p, d_scratch, a);
    } else {
        const double *p = (const double *)st;
        if (nt <= 8)
            hipLaunchKernelGGL((k_expect_z<double, 8>), g, b, 0, s, p, d_scratch, a);
        else if (nt <= 16)
            hipLaunchKernelGGL((k_expect_z<double, 16>), g, b, 0, s, p, d_scratch, a);
        else
            hipLaunchKernelGGL((k_expect_z<double, 32>), g, b, 0, s, p, d_scratch, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_sum_rows(d_scratch, d_out, uint64_t(nt), grid, s);
}

hipError_t launch_expect_xy(const void *st, int n, int dtype, uint64_t xmask, uint64_t yzmask, double *d_scratch,
                            double *d_out2, hipStream_t s)
{
    if (xmask == 0)
        return hipErrorInvalidValue;
    ExpXYArgs a{};
    int h = 63 - __builtin_clzll(xmask);
    a.hmask = (uint64_t(1) << h) - 1;
    a.x = xmask;
    a.yz = yzmask;
    a.npairs = uint64_t(1) << (n - 1);
    const uint32_t grid = exp_grid(n - 1);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_expect_xy<float>, dim3(grid), dim3(kThreads), 0, s, (const float *)st, d_scratch, a);
    else
        hipLaunchKernelGGL(k_expect_xy<double>, dim3(grid), dim3(kThreads), 0, s, (const double *)st, d_scratch, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_sum_rows(d_scratch, d_out2, uint64_t(2), grid, s);
}

int sample_log_block(int n)
{
    return n < 14 ? n : 14;
}

hipError_t launch_block_sums(const void *st, int n, int dtype, double *d_bsums, hipStream_t s)
{
    const int lbs = sample_log_block(n);
    const uint64_t nb = uint64_t(1) << (n - lbs);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_block_sums<float>, dim3(uint32_t(nb)), dim3(kThreads), 0, s, (const float *)st, d_bsums, lbs);
    else
        hipLaunchKernelGGL(k_block_sums<double>, dim3(uint32_t(nb)), dim3(kThreads), 0, s, (const double *)st, d_bsums, lbs);
    return hipGetLastError();
}

hipError_t launch_sample_prep(const double *d_bsums, uint64_t nb, const double *d_uniforms, int shots,
                              int64_t *d_blocks, double *d_targets, hipStream_t s)
{
    if (shots <= 0)
        return hipSuccess;
    if (nb == 0 || (nb & (nb - 1)) != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample_prep, dim3(1), dim3(kPrepThreads), 0, s, d_bsums, nb, d_uniforms, shots, d_blocks,
                       d_targets);
    return hipGetLastError();
}

hipError_t launch_sample_search(const void *st, int n, int dtype, const int64_t *d_blocks, const double *d_targets,
                                int shots, int64_t *d_out, int lbs, hipStream_t s)
{
    if (shots <= 0 || lbs < 1 || lbs > n || lbs > 20)
        return hipSuccess;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_sample_search<float>, dim3(shots), dim3(kThreads), 0, s, (const float *)st, d_blocks,
                           d_targets, d_out, lbs);
    else
        hipLaunchKernelGGL(k_sample_search<double>, dim3(shots), dim3(kThreads), 0, s, (const double *)st, d_blocks,
                           d_targets, d_out, lbs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused read-out: one k_marg_fold launch over the state gives the marginal's
// fold (when it takes the register-summed fold route), the partial sums of up
// to kMaxZ Z strings and the block totals for sampling; then the marginal's
// second stage and the Z reduction.
// ---------------------------------------------------------------------------
namespace {

// Route of the fused launch; false where the marginal takes another route.
// m = 0: a fold with no bin bits (the total only).
// More segments per workgroup than the marginal alone needs: at most 2^12
// workgroups, so that the per-workgroup reductions of the Z strings (one per
// string) and the partial sums they leave stay small against the read.
bool fused_route(int n, int m, const int *phys_q, int dtype, MargRoute &r)
{
    if (n < kSegLog + 2)
        return false;
    int F = 0;
    uint64_t hibins = 0;
    if (m > 0) {
        r = marg_route(n, m, phys_q);
        if (r.kind != 2)
            return false;
        const int low = dtype == SV_C64 ? fold_low_bits<float>() : fold_low_bits<double>();
        if ((r.fold.binmask >> low) != 0)
            return false;
        F = r.fold.F;
        for (int b = 0; b < m; ++b)
            if (phys_q[b] >= kSegLog)
                hibins |= uint64_t(1) << phys_q[b];
    }
    const int want = std::max(0, n - kSegLog - 12);
    while (F < want && F < n - kSegLog - 1 && !((hibins >> (kSegLog + F)) & 1))
        ++F;
    while (F < n - kSegLog - 1 && !((hibins >> (kSegLog + F)) & 1) &&
           (uint64_t(1) << (n - kSegLog - F)) > kMaxFolded)
        ++F;
    r = fold_route(n, m, phys_q, F);
    return true;
}

}  // namespace

static_assert(kMaxZ == kReadoutMaxZ, "Z strings of one fused read-out");

bool readout_fusable(int n, int m, const int *phys_q, int dtype)
{
    MargRoute r;
    return fused_route(n, m, phys_q, dtype, r);
}

int readout_log_block(int n, int m, const int *phys_q, int dtype)
{
    MargRoute r;
    if (!fused_route(n, m, phys_q, dtype, r))
        return -1;
    return kSegLog + std::min(r.fold.F, 2);
}

uint64_t readout_scratch_doubles(int n, int m, const int *phys_q, int dtype)
{
    MargRoute r;
    if (!fused_route(n, m, phys_q, dtype, r))
        return 0;
    const uint64_t nblk = uint64_t(1) << (n - kSegLog - r.fold.F);
    return r.scratch + uint64_t(kMaxZ) * nblk;
}

hipError_t launch_readout(const void *st, int n, int dtype, const int *phys_q, int m, const uint64_t *zmasks,
                          int nt, double *d_scratch, double *d_marg, double *d_z, double *d_tot, hipStream_t s)
{
    MargRoute r;
    if (nt < 0 || nt > kMaxZ || !fused_route(n, m, phys_q, dtype, r))
        return hipErrorInvalidValue;
    const uint64_t nblk = uint64_t(1) << (n - kSegLog - r.fold.F);
    ReadoutArgs ra{};
    ra.nt = nt;
    for (int t = 0; t < nt; ++t)
        ra.z[t] = zmasks[t];
    ra.tlog = std::min(r.fold.F, 2);
    ra.zpart = d_scratch + r.scratch;
    ra.tot = d_tot;
    const dim3 g{uint32_t(nblk)}, b{uint32_t(kThreads)};
    if (dtype == SV_C64) {
        const float *p = (const float *)st;
        if (nt > 0)
            hipLaunchKernelGGL((k_marg_fold<float, true, kMaxZ, true>), g, b, 0, s, p, d_scratch, r.fold, ra);
        else
            hipLaunchKernelGGL((k_marg_fold<float, true, 0, true>), g, b, 0, s, p, d_scratch, r.fold, ra);
    } else {
        const double *p = (const double *)st;
        if (nt > 0)
            hipLaunchKernelGGL((k_marg_fold<double, true, kMaxZ, true>), g, b, 0, s, p, d_scratch, r.fold, ra);
        else
            hipLaunchKernelGGL((k_marg_fold<double, true, 0, true>), g, b, 0, s, p, d_scratch, r.fold, ra);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (nt > 0) {
        e = launch_sum_rows(ra.zpart, d_z, uint64_t(nt), uint32_t(nblk), s);
        if (e != hipSuccess)
            return e;
    }
    if (m == 0 || !d_marg)
        return hipSuccess;
    MargArgs a2{};
    a2.m = m;
    a2.rest = uint64_t(1) << (r.n2 - m);
    a2.nbins = uint32_t(1u << m);
    for (int b2 = 0; b2 < m; ++b2)
        a2.qbit[b2] = uint64_t(1) << r.q2[size_t(b2)];
    a2.rest_im = make_masks(r.q2);
    a2.chunks = r.p2.chunks;
    a2.per_chunk = r.p2.per_chunk;
    if (r.p2.rmajor) {
        double *part = d_scratch + r.red;
        hipLaunchKernelGGL(k_marg_rmajor_d, dim3(a2.chunks, a2.nbins), dim3(kThreads), 0, s, d_scratch, part, a2);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        return launch_sum_rows(part, d_marg, uint64_t(a2.nbins), a2.chunks, s);
    }
    const uint64_t gg = std::min<uint64_t>((uint64_t(a2.nbins) + kThreads - 1) / kThreads, 1u << 20);
    hipLaunchKernelGGL(k_marg_doubles, dim3(gg), dim3(kThreads), 0, s, d_scratch, d_marg, a2);
    return hipGetLastError();
}

}  // namespace sv
