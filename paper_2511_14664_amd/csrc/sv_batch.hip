// Persistent batch kernel: many small circuits in one launch (gfx950).
//
// Workgroups take tasks (circuit, pass, tile) from a global queue in a fixed
// order.  A task loads its tile of 2^lp amplitudes into LDS (or creates
// |0...0> for the first pass), applies the pass's gates in LDS -- each one a
// sweep over the tile, paper Sec. 2.1 -- and either stores the tile or, on the
// last pass, reduces the Z-string expectation values of its amplitudes in
// FP64.  A task of pass p waits until every tile of passes < p of its circuit
// is done; those tasks were dequeued earlier by resident workgroups, so the
// wait always ends.  The wait is still bounded: past the spin limit the task
// raises the error flag, every workgroup drains, and the host reports it.
//
// Cross-workgroup visibility: every thread issues an agent-scope release
// fence after its stores (L2 write-back and wait), then a barrier, then one
// atomic increment; a consumer reads the count, passes a barrier, and every
// thread issues an agent-scope acquire fence before loading.
#include "sv_batch.h"
#include "sv_device.h"

namespace sv {
namespace {

using namespace dev;

__device__ __forceinline__ uint32_t ins1(uint32_t j, int a)
{
    return (j & ((1u << a) - 1u)) | ((j >> a) << (a + 1));
}

// Insert zeros at tile bits lo < hi.
__device__ __forceinline__ uint32_t ins2(uint32_t j, int lo, int hi)
{
    return ins1(ins1(j, lo), hi);
}

// acc + u * v as four fused multiply-adds (the state arithmetic of the
// in-LDS sweeps; every product is rounded once, into the running sum)
__device__ __forceinline__ float fma_r(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fma_r(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}
template <typename C>
__device__ __forceinline__ C cfma(C u, C v, C acc)
{
    acc.x = fma_r(u.x, v.x, acc.x);
    acc.x = fma_r(-u.y, v.y, acc.x);
    acc.y = fma_r(u.x, v.y, acc.y);
    acc.y = fma_r(u.y, v.x, acc.y);
    return acc;
}

// Element of the LDS tile at byte offset o.  swz() is linear over XOR, so
// the offsets of a group's members are one XOR away from its first one.
template <typename C>
__device__ __forceinline__ C &lds_at(unsigned char *tileb, uint32_t o)
{
    return *reinterpret_cast<C *>(tileb + o);
}

// Agent-scope release of this wave's global stores, completed before the
// wave goes on: the compiler may otherwise leave the write-back's wait for the
// next atomic, which only one wave of the workgroup issues.
__device__ __forceinline__ void publish()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);  // vmcnt, expcnt and lgkmcnt all zero
}

// Device-scope store of one amplitude (relaxed atomic 64-bit stores): the
// write goes through the XCD's L2, so the release after the tile finds no
// dirty lines of it there to write back.
template <typename C>
__device__ __forceinline__ void store_dev(C *p, C v)
{
    static_assert(sizeof(C) % 8 == 0, "amplitudes of 8 or 16 bytes");
    uint64_t w[sizeof(C) / 8];
    __builtin_memcpy(w, &v, sizeof(C));
    uint64_t *q = reinterpret_cast<uint64_t *>(p);
#pragma unroll
    for (size_t i = 0; i < sizeof(C) / 8; ++i)
        __hip_atomic_store(q + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <typename R>
__global__ __launch_bounds__(kBatchThreads) void k_batch(const BatchArgs a)
{
    using C = typename CT<R>::C;
    // tile amplitudes per thread in flight between global memory and LDS
    constexpr uint32_t kU = 8;
    typedef R VU __attribute__((ext_vector_type(2 * kU)));
    extern __shared__ __align__(16) unsigned char smem[];
    C *tile = reinterpret_cast<C *>(smem);
    unsigned char *tileb = smem;
    double *red = reinterpret_cast<double *>(smem + (sizeof(C) << a.tile_log_max));  // [waves][16]
    C *mcache = reinterpret_cast<C *>(red + (kBatchThreads / 64) * 16);
    BStep *scache = reinterpret_cast<BStep *>(reinterpret_cast<unsigned char *>(mcache) + kBatchMatCacheBytes);
    constexpr uint32_t kMatCap = kBatchMatCacheBytes / sizeof(C);
    __shared__ uint32_t s_task;
    __shared__ int s_flag;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t *head = a.ctr;
    uint32_t *err = a.ctr + 1;
    uint32_t *done = a.ctr + 2;
    uint32_t *fin = a.ctr + 2 + a.ninst;
    C *states = reinterpret_cast<C *>(a.states);
    const C *mats = reinterpret_cast<const C *>(a.mats);

    for (;;) {
        if (tid == 0) {
            uint32_t t = atomicAdd(head, 1u);
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                t = a.ntasks;
            s_task = t;
        }
        __syncthreads();
        const uint32_t t = s_task;
        if (t >= a.ntasks)
            break;
        const BTask tk = a.tasks[t];
        const BInst in = a.inst[tk.inst];
        const BPass &ps = a.pass[in.pass0 + int(tk.pass)];
        const int lp = ps.lp;
        const uint32_t TA = 1u << lp;

        if (tk.pass > 0) {
            if (tid == 0) {
                int ok = 1;
                uint32_t spins = 0;
                while (__hip_atomic_load(&done[tk.inst], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < ps.need) {
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        ++spins > a.spin_limit) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                if (!ok)
                    atomicOr(err, 1u);
                s_flag = ok;
            }
            __syncthreads();
            if (!s_flag)
                break;
            // pairs with the producers' release (the count was read relaxed)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }

        // the pass's steps and matrices into LDS (visible after the barrier
        // that ends the tile load; the previous task's last reads of them
        // ended at its final barrier)
        const bool cached = ps.nsteps <= kBatchStepCache && ps.nmat <= kMatCap;
        if (cached) {
            for (int i = tid; i < ps.nsteps; i += kBatchThreads)
                scache[i] = a.steps[ps.step0 + i];
            for (uint32_t i = tid; i < ps.nmat; i += kBatchThreads)
                mcache[i] = mats[ps.mat0 + i];
        }

        // tile index -> base, and per-thread low part of the tile offsets
        uint64_t base = tk.tile;
        for (int b = 0; b < lp; ++b) {
            const uint64_t m = ps.ins[b];
            base = (base & m) | ((base & ~m) << 1);
        }
        uint64_t off_lo = 0;
        for (int b = 0; b < kBatchThreadLog && b < lp; ++b)
            if ((tid >> b) & 1)
                off_lo |= ps.dep[b];
        // deposits of the tile bits above the thread bits in registers: the
        // pass table is not re-read after every store of the tile
        constexpr int kHi = kBatchMaxTileLog - kBatchThreadLog;
        uint64_t dep_hi[kHi];
#pragma unroll
        for (int b = 0; b < kHi; ++b)
            dep_hi[b] = b + kBatchThreadLog < lp ? ps.dep[b + kBatchThreadLog] : 0;
        auto off_of = [&](uint32_t s) {
            uint64_t off = off_lo;
#pragma unroll
            for (int b = 0; b < kHi; ++b)
                if ((s >> b) & 1)
                    off |= dep_hi[b];
            return off;
        };
        const uint32_t nsteps_x = TA >= kBatchThreads ? TA / kBatchThreads : 1;
        const bool active = uint32_t(tid) < TA;
        C *st = states + in.state_off;

        if (tk.pass == 0) {
            for (uint32_t s = 0; s < nsteps_x; ++s) {
                if (!active)
                    break;
                const uint32_t x = s * kBatchThreads + uint32_t(tid);
                C z;
                z.x = (tk.tile == 0 && x == 0) ? R(1) : R(0);
                z.y = R(0);
                tile[swz(x)] = z;
            }
        } else if (nsteps_x >= kU) {
            // kU global loads in flight per thread before the first LDS store
            // (nsteps_x and kU are powers of two: whole chunks)
            for (uint32_t s0 = 0; s0 < nsteps_x; s0 += kU) {
                VU v;  // a vector, not an array: stays in registers
#pragma unroll
                for (uint32_t u = 0; u < kU; ++u) {
                    const C x = st[base + off_of(s0 + u)];
                    v[2 * u] = x.x;
                    v[2 * u + 1] = x.y;
                }
#pragma unroll
                for (uint32_t u = 0; u < kU; ++u) {
                    C x;
                    x.x = v[2 * u];
                    x.y = v[2 * u + 1];
                    tile[swz((s0 + u) * kBatchThreads + uint32_t(tid))] = x;
                }
            }
        } else {
            for (uint32_t s = 0; s < nsteps_x; ++s) {
                if (!active)
                    break;
                tile[swz(s * kBatchThreads + uint32_t(tid))] = st[base + off_of(s)];
            }
        }
        __syncthreads();

        // the steps, reading step records and matrices from the LDS copies
        // (LDS) or from global memory (false)
        auto sweeps = [&](auto lds_tag) __attribute__((always_inline)) {
          constexpr bool kLds = decltype(lds_tag)::value;
          for (int si = 0; si < ps.nsteps; ++si) {
            BStep sp;
            if constexpr (kLds)
                sp = scache[si];
            else
                sp = a.steps[ps.step0 + si];
            const C *M = kLds ? mcache + (sp.mat - ps.mat0) : mats + sp.mat;
            const int ta = sp.a, tb = sp.b;
            // Each sweep takes one group per thread per iteration (two or four
            // groups with all their LDS reads ahead were slower).
            if (sp.type <= 1) {
                const C m00 = M[0], m01 = M[1], m10 = M[2], m11 = M[3];
                const int lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
                const bool ctl = sp.type == 1;
                const uint32_t cnt = ctl ? TA / 4 : TA / 2;
                const uint32_t cbit = ctl ? 1u << tb : 0u;
                const uint32_t pt = swz(1u << ta) * uint32_t(sizeof(C));  // partner: byte offset XOR
                auto first = [&](uint32_t j) __attribute__((always_inline)) {
                    return swz((ctl ? ins2(j, lo, hi) : ins1(j, ta)) | cbit) * uint32_t(sizeof(C));
                };
                for (uint32_t j = tid; j < cnt; j += kBatchThreads) {
                    const uint32_t o = first(j);
                    const C v0 = lds_at<C>(tileb, o), v1 = lds_at<C>(tileb, o ^ pt);
                    lds_at<C>(tileb, o) = cfma(m01, v1, cmul(m00, v0));
                    lds_at<C>(tileb, o ^ pt) = cfma(m11, v1, cmul(m10, v0));
                }
            } else {
                C m[16];
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    m[e] = M[e];
                const int lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
                const uint32_t cnt = TA / 4;
                // byte-offset XORs of the group members (matrix index e:
                // bit 0 on tile bit ta, bit 1 on tile bit tb)
                uint32_t px[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    px[e] = swz(((e & 1) ? 1u << ta : 0u) | ((e & 2) ? 1u << tb : 0u)) * uint32_t(sizeof(C));
                for (uint32_t j = tid; j < cnt; j += kBatchThreads) {
                    const uint32_t o = swz(ins2(j, lo, hi)) * uint32_t(sizeof(C));
                    C v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        v[e] = lds_at<C>(tileb, o ^ px[e]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        C acc = cmul(m[r * 4], v[0]);
#pragma unroll
                        for (int c = 1; c < 4; ++c)
                            acc = cfma(m[r * 4 + c], v[c], acc);
                        lds_at<C>(tileb, o ^ px[r]) = acc;
                    }
                }
            }
            __syncthreads();
          }
        };
        if (cached)
            sweeps(std::true_type{});
        else
            sweeps(std::false_type{});

        if (!ps.last) {
            if (nsteps_x >= kU) {
                for (uint32_t s0 = 0; s0 < nsteps_x; s0 += kU) {
                    VU v;
#pragma unroll
                    for (uint32_t u = 0; u < kU; ++u) {
                        const C x = tile[swz((s0 + u) * kBatchThreads + uint32_t(tid))];
                        v[2 * u] = x.x;
                        v[2 * u + 1] = x.y;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kU; ++u) {
                        C x;
                        x.x = v[2 * u];
                        x.y = v[2 * u + 1];
                        store_dev(&st[base + off_of(s0 + u)], x);
                    }
                }
            } else {
                for (uint32_t s = 0; s < nsteps_x; ++s) {
                    if (!active)
                        break;
                    store_dev(&st[base + off_of(s)], tile[swz(s * kBatchThreads + uint32_t(tid))]);
                }
            }
            // Every wave writes its stores back past L2 (an agent-scope release:
            // write-back, no invalidate) and waits for the write-back before
            // the barrier; then one thread raises the count.
            publish();
            __syncthreads();
            if (tid == 0)
                __hip_atomic_fetch_add(&done[tk.inst], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t *zm = a.zmasks + in.term0;
            for (int c0 = 0; c0 < in.nterms; c0 += 16) {
                double acc[16];
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    acc[j] = 0.0;
                for (uint32_t s = 0; s < nsteps_x; ++s) {
                    if (!active)
                        break;
                    const uint32_t x = s * kBatchThreads + uint32_t(tid);
                    const uint64_t gi = base + off_of(s);
                    const C v = tile[swz(x)];
                    const double p = double(v.x) * double(v.x) + double(v.y) * double(v.y);
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if (c0 + j < in.nterms)
                            acc[j] += (__popcll(gi & zm[c0 + j]) & 1) ? -p : p;
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const double w = wave_sum(acc[j]);
                    if (lane == 0)
                        red[wave * 16 + j] = w;
                }
                __syncthreads();
                if (tid < 16 && c0 + tid < in.nterms) {
                    double v = red[tid];
#pragma unroll
                    for (int w = 1; w < kBatchThreads / 64; ++w)
                        v += red[16 * w + tid];
                    if (ps.ntiles == 1)
                        a.out[in.out0 + c0 + tid] = v;
                    else
                        a.partials[in.part0 + size_t(tk.tile) * in.nterms + c0 + tid] = v;
                }
                __syncthreads();
            }
            if (ps.ntiles > 1) {
                publish();
                __syncthreads();
                if (tid == 0)
                    s_flag = __hip_atomic_fetch_add(&fin[tk.inst], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                             ps.ntiles - 1;
                __syncthreads();
                if (s_flag) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    for (int j = tid; j < in.nterms; j += kBatchThreads) {
                        double sum = 0.0;
                        for (uint32_t tl = 0; tl < ps.ntiles; ++tl)
                            sum += __hip_atomic_load(&a.partials[in.part0 + size_t(tl) * in.nterms + j],
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        a.out[in.out0 + j] = sum;
                    }
                }
            }
        }
        __syncthreads();
    }
}

__global__ void k_batch_fill(uint32_t *ctr, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ctr[i] = 0u;
}

}  // namespace

hipError_t launch_batch(int dtype, const BatchArgs &a, uint32_t grid, size_t lds, hipStream_t s)
{
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(kBatchThreads), lds, s, a);
    else
        hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(kBatchThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_fill(uint32_t *ctr, uint32_t n, hipStream_t s)
{
    const uint32_t grid = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_batch_fill, dim3(grid < 1 ? 1 : grid), dim3(kThreads), 0, s, ctr, n);
    return hipGetLastError();
}

uint32_t batch_grid(int dtype, size_t lds)
{
    const void *k = dtype == SV_C64 ? reinterpret_cast<const void *>(&k_batch<float>)
                                    : reinterpret_cast<const void *>(&k_batch<double>);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBatchThreads, lds) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    return uint32_t(cus * per_cu);
}

}  // namespace sv
