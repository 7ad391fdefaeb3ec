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
// Cross-workgroup visibility uses agent-scope release (every thread fences
// its own stores, then one atomic increment) and acquire (atomic load, then an
// agent-scope acquire fence in every thread).
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

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_batch(const BatchArgs a)
{
    using C = typename CT<R>::C;
    extern __shared__ __align__(16) unsigned char smem[];
    C *tile = reinterpret_cast<C *>(smem);
    double *red = reinterpret_cast<double *>(smem + (sizeof(C) << a.tile_log_max));  // [4][16]
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
                while (__hip_atomic_load(&done[tk.inst], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < ps.need) {
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
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }

        // tile index -> base, and per-thread low part of the tile offsets
        uint64_t base = tk.tile;
        for (int b = 0; b < lp; ++b) {
            const uint64_t m = ps.ins[b];
            base = (base & m) | ((base & ~m) << 1);
        }
        uint64_t off_lo = 0;
        for (int b = 0; b < 8 && b < lp; ++b)
            if ((tid >> b) & 1)
                off_lo |= ps.dep[b];
        auto off_of = [&](uint32_t s) {
            uint64_t off = off_lo;
            for (int b = 8; b < lp; ++b)
                if ((s >> (b - 8)) & 1)
                    off |= ps.dep[b];
            return off;
        };
        const uint32_t nsteps_x = TA >= kThreads ? TA / kThreads : 1;
        const bool active = uint32_t(tid) < TA;
        C *st = states + in.state_off;

        if (tk.pass == 0) {
            for (uint32_t s = 0; s < nsteps_x; ++s) {
                if (!active)
                    break;
                const uint32_t x = s * kThreads + uint32_t(tid);
                C z;
                z.x = (tk.tile == 0 && x == 0) ? R(1) : R(0);
                z.y = R(0);
                tile[swz(x)] = z;
            }
        } else {
            for (uint32_t s = 0; s < nsteps_x; ++s) {
                if (!active)
                    break;
                tile[swz(s * kThreads + uint32_t(tid))] = st[base + off_of(s)];
            }
        }
        __syncthreads();

        for (int si = 0; si < ps.nsteps; ++si) {
            const BStep sp = a.steps[ps.step0 + si];
            const C *M = mats + sp.mat;
            const int ta = sp.a, tb = sp.b;
            if (sp.type == 0) {
                const C m00 = M[0], m01 = M[1], m10 = M[2], m11 = M[3];
                for (uint32_t j = tid; j < TA / 2; j += kThreads) {
                    const uint32_t x0 = ins1(j, ta), x1 = x0 | (1u << ta);
                    const C v0 = tile[swz(x0)], v1 = tile[swz(x1)];
                    tile[swz(x0)] = cmad(m01, v1, cmul(m00, v0));
                    tile[swz(x1)] = cmad(m11, v1, cmul(m10, v0));
                }
            } else if (sp.type == 1) {
                const C m00 = M[0], m01 = M[1], m10 = M[2], m11 = M[3];
                const int lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
                for (uint32_t j = tid; j < TA / 4; j += kThreads) {
                    const uint32_t x0 = ins2(j, lo, hi) | (1u << tb), x1 = x0 | (1u << ta);
                    const C v0 = tile[swz(x0)], v1 = tile[swz(x1)];
                    tile[swz(x0)] = cmad(m01, v1, cmul(m00, v0));
                    tile[swz(x1)] = cmad(m11, v1, cmul(m10, v0));
                }
            } else {
                C m[16];
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    m[e] = M[e];
                const int lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
                for (uint32_t j = tid; j < TA / 4; j += kThreads) {
                    const uint32_t b0 = ins2(j, lo, hi);
                    uint32_t xi[4];
                    C v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        xi[e] = b0 | (uint32_t(e & 1) << ta) | (uint32_t(e >> 1) << tb);
                        v[e] = tile[swz(xi[e])];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        C acc = czero<C>();
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            acc = cmad(m[r * 4 + c], v[c], acc);
                        tile[swz(xi[r])] = acc;
                    }
                }
            }
            __syncthreads();
        }

        if (!ps.last) {
            for (uint32_t s = 0; s < nsteps_x; ++s) {
                if (!active)
                    break;
                st[base + off_of(s)] = tile[swz(s * kThreads + uint32_t(tid))];
            }
            __threadfence();
            __syncthreads();
            if (tid == 0)
                atomicAdd(&done[tk.inst], 1u);
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
                    const uint32_t x = s * kThreads + uint32_t(tid);
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
                    const double v = ((red[tid] + red[16 + tid]) + red[32 + tid]) + red[48 + tid];
                    if (ps.ntiles == 1)
                        a.out[in.out0 + c0 + tid] = v;
                    else
                        a.partials[in.part0 + size_t(tk.tile) * in.nterms + c0 + tid] = v;
                }
                __syncthreads();
            }
            if (ps.ntiles > 1) {
                __threadfence();
                __syncthreads();
                if (tid == 0)
                    s_flag = atomicAdd(&fin[tk.inst], 1u) == ps.ntiles - 1;
                __syncthreads();
                if (s_flag) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    for (int j = tid; j < in.nterms; j += kThreads) {
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
        hipLaunchKernelGGL(k_batch<float>, dim3(grid), dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL(k_batch<double>, dim3(grid), dim3(kThreads), lds, s, a);
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, lds) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    return uint32_t(cus * per_cu);
}

}  // namespace sv
