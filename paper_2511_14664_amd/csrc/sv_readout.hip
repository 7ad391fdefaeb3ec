// Read-out sweeps: marginal probabilities, Pauli expectation values and
// sampling (paper Sec. 2.1 "Measurement and Sampling", shots of Sec. 2.2).
// Each is one read pass over the state; all accumulation is FP64 whatever the
// amplitude precision, with a fixed reduction order (no atomics), so results
// are reproducible run to run.
#include <algorithm>
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

// ---------------------------------------------------------------------------
// Z-string expectations: sum_i |a_i|^2 (-1)^popcount(i & z_t), up to 16
// strings per pass.  part[t * gridDim + block].
// ---------------------------------------------------------------------------
constexpr int kMaxZ = 16;
struct ExpZArgs {
    uint64_t nelem;
    int nt;
    uint64_t z[kMaxZ];
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_expect_z(const R *__restrict__ st, double *__restrict__ part,
                                                       const ExpZArgs a)
{
    using C = typename CT<R>::C;
    __shared__ double sh[4];
    const C *v = reinterpret_cast<const C *>(st);
    double acc[kMaxZ];
#pragma unroll
    for (int t = 0; t < kMaxZ; ++t)
        acc[t] = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kThreads;
    // four independent loads in flight per thread
    for (uint64_t i0 = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i0 < a.nelem; i0 += 4 * stride) {
        double p[4];
        uint64_t ii[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ii[u] = i0 + uint64_t(u) * stride;
            p[u] = ii[u] < a.nelem ? prob(v[ii[u]]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < kMaxZ; ++t)
                if (t < a.nt)
                    acc[t] += (__popcll(ii[u] & a.z[t]) & 1) ? -p[u] : p[u];
    }
#pragma unroll
    for (int t = 0; t < kMaxZ; ++t) {
        if (t < a.nt) {
            const double s = block_sum(acc[t], sh);
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
template <typename R>
__global__ __launch_bounds__(kThreads) void k_block_sums(const R *__restrict__ st, double *__restrict__ bs,
                                                         int lbs)
{
    using C = typename CT<R>::C;
    __shared__ double sh[4];
    const C *v = reinterpret_cast<const C *>(st);
    const uint64_t base = uint64_t(blockIdx.x) << lbs;
    const uint32_t bsz = 1u << lbs;
    double acc = 0.0;
    for (uint32_t e = threadIdx.x; e < bsz; e += kThreads)
        acc += prob(v[base + e]);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0)
        bs[blockIdx.x] = acc;
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

uint64_t marginal_scratch_doubles(int n, int m)
{
    MargPlan p = marg_plan(n, m);
    const uint64_t old = p.rmajor ? (uint64_t(1) << m) * p.chunks : 1;
    const uint64_t seg = n >= 12 ? (uint64_t(1) << (n - 12)) : 1;
    return std::max(old, seg);
}

hipError_t launch_marginal(const void *st, int n, int dtype, const int *phys_q, int m, double *d_scratch,
                           double *d_out, hipStream_t s)
{
    if (m < 0 || m > kMaxQ || m > n)
        return hipErrorInvalidValue;
    // segment path: every bin bit at or above bit 12
    int b0 = n;
    for (int b = 0; b < m; ++b)
        b0 = std::min(b0, phys_q[b]);
    if (n >= 12 && b0 >= 12) {
        const int sb = std::min(b0, 16);
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
        const uint64_t g = (uint64_t(a.nbins) + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_sum_rows, dim3(g), dim3(kThreads), 0, s, d_scratch, d_out, uint64_t(a.nbins),
                           p.chunks);
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

uint64_t expect_scratch_doubles(int n)
{
    (void)n;
    return uint64_t(kMaxZ) * kExpGrid;
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
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_expect_z<float>, dim3(grid), dim3(kThreads), 0, s, (const float *)st, d_scratch, a);
    else
        hipLaunchKernelGGL(k_expect_z<double>, dim3(grid), dim3(kThreads), 0, s, (const double *)st, d_scratch, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kThreads), 0, s, d_scratch, d_out, uint64_t(nt), grid);
    return hipGetLastError();
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
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kThreads), 0, s, d_scratch, d_out2, uint64_t(2), grid);
    return hipGetLastError();
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

hipError_t launch_sample_search(const void *st, int n, int dtype, const int64_t *d_blocks, const double *d_targets,
                                int shots, int64_t *d_out, hipStream_t s)
{
    const int lbs = sample_log_block(n);
    if (shots <= 0)
        return hipSuccess;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_sample_search<float>, dim3(shots), dim3(kThreads), 0, s, (const float *)st, d_blocks,
                           d_targets, d_out, lbs);
    else
        hipLaunchKernelGGL(k_sample_search<double>, dim3(shots), dim3(kThreads), 0, s, (const double *)st, d_blocks,
                           d_targets, d_out, lbs);
    return hipGetLastError();
}

}  // namespace sv
