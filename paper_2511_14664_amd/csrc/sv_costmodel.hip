// Learned sweep cost model: a 10-64-64-1 ReLU network trained on the GPU on
// sweep timings the library measures itself, used to rank fusion plans.
//
// Training: one workgroup of 64 threads (one per hidden unit) per chunk of
// samples runs forward and backward in FP32 and accumulates its chunk's
// gradient in registers; a second kernel sums the chunk partials in a fixed
// order and applies Adam.  Inference: weights and activations in FP16, dot
// products by v_dot2_f32_f16 with FP32 accumulation, one thread per sample.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sv_internal.h"

namespace sv {
namespace {

constexpr int F = SV_CM_FEATURES;
constexpr int H = SV_CM_HIDDEN;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * F;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
constexpr int P = OFF_B3 + 1;
constexpr int PS = P + 1;  // partial stride: gradient + loss
constexpr int kMaxChunks = 64;

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(H) void k_mlp_grad(const float *__restrict__ prm, const float *__restrict__ x,
                                                const float *__restrict__ y, int n, float two_over_n,
                                                float *__restrict__ part)
{
    __shared__ float W2s[H][H + 1];
    __shared__ float h1s[H], dh2s[H], xs[F];
    const int j = threadIdx.x;
    float w1[F];
#pragma unroll
    for (int f = 0; f < F; ++f)
        w1[f] = prm[OFF_W1 + j * F + f];
    const float b1 = prm[OFF_B1 + j], b2 = prm[OFF_B2 + j], w3 = prm[OFF_W3 + j], b3 = prm[OFF_B3];
    for (int i = 0; i < H; ++i)
        W2s[j][i] = prm[OFF_W2 + j * H + i];
    float gw1[F], gw2[H];
#pragma unroll
    for (int f = 0; f < F; ++f)
        gw1[f] = 0.0f;
#pragma unroll
    for (int i = 0; i < H; ++i)
        gw2[i] = 0.0f;
    float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
    __syncthreads();
    for (int s = blockIdx.x; s < n; s += gridDim.x) {
        if (j < F)
            xs[j] = x[size_t(s) * F + j];
        __syncthreads();
        float a1 = b1;
#pragma unroll
        for (int f = 0; f < F; ++f)
            a1 += w1[f] * xs[f];
        h1s[j] = a1 > 0.0f ? a1 : 0.0f;
        __syncthreads();
        float a2 = b2;
#pragma unroll
        for (int i = 0; i < H; ++i)
            a2 += W2s[j][i] * h1s[i];
        const float h2 = a2 > 0.0f ? a2 : 0.0f;
        float yv = w3 * h2;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            yv += __shfl_xor(yv, off, 64);
        yv += b3;
        const float r = yv - y[s];
        const float dout = two_over_n * r;
        if (j == 0) {
            lsum += r * r;
            gb3 += dout;
        }
        gw3 += dout * h2;
        const float dh2 = a2 > 0.0f ? dout * w3 : 0.0f;
        gb2 += dh2;
#pragma unroll
        for (int i = 0; i < H; ++i)
            gw2[i] += dh2 * h1s[i];
        dh2s[j] = dh2;
        __syncthreads();
        float dh1 = 0.0f;
#pragma unroll
        for (int k = 0; k < H; ++k)
            dh1 += dh2s[k] * W2s[k][j];
        dh1 = a1 > 0.0f ? dh1 : 0.0f;
        gb1 += dh1;
#pragma unroll
        for (int f = 0; f < F; ++f)
            gw1[f] += dh1 * xs[f];
        __syncthreads();
    }
    float *pp = part + size_t(blockIdx.x) * PS;
#pragma unroll
    for (int f = 0; f < F; ++f)
        pp[OFF_W1 + j * F + f] = gw1[f];
    pp[OFF_B1 + j] = gb1;
#pragma unroll
    for (int i = 0; i < H; ++i)
        pp[OFF_W2 + j * H + i] = gw2[i];
    pp[OFF_B2 + j] = gb2;
    pp[OFF_W3 + j] = gw3;
    if (j == 0) {
        pp[OFF_B3] = gb3;
        pp[P] = lsum;
    }
}

// Sum chunk partials (ascending chunk); mode 0: write gradient, 1: Adam step.
__global__ __launch_bounds__(256) void k_mlp_update(float *__restrict__ prm, float *__restrict__ m,
                                                    float *__restrict__ v, const float *__restrict__ part,
                                                    int chunks, int mode, float lr, float c1, float c2,
                                                    float inv_n, float *__restrict__ grad_out,
                                                    float *__restrict__ loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P)
        return;
    float g = 0.0f;
    for (int c = 0; c < chunks; ++c)
        g += part[size_t(c) * PS + p];
    if (p == P) {
        *loss_out = g * inv_n;
        return;
    }
    if (mode == 0) {
        grad_out[p] = g;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    // c1 = 1 - b1^t, c2 = 1 - b2^t (bias corrections)
    prm[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_to_half(const float *__restrict__ prm, _Float16 *__restrict__ ph)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P)
        ph[p] = _Float16(prm[p]);
}

// One thread per sample.  Weights in LDS (FP16), dot products of FP16 pairs
// accumulated in FP32.
__global__ __launch_bounds__(256) void k_mlp_predict(const _Float16 *__restrict__ ph, const float *__restrict__ x,
                                                     int n, float *__restrict__ out)
{
    __shared__ half2v W1s[H][F / 2];
    __shared__ half2v W2s[H][H / 2];
    __shared__ float b1s[H], b2s[H], w3s[H];
    __shared__ float b3s;
    for (int e = threadIdx.x; e < H * F / 2; e += blockDim.x) {
        const int r = e / (F / 2), c = e % (F / 2);
        half2v w;
        w.x = ph[OFF_W1 + r * F + 2 * c];
        w.y = ph[OFF_W1 + r * F + 2 * c + 1];
        W1s[r][c] = w;
    }
    for (int e = threadIdx.x; e < H * H / 2; e += blockDim.x) {
        const int r = e / (H / 2), c = e % (H / 2);
        half2v w;
        w.x = ph[OFF_W2 + r * H + 2 * c];
        w.y = ph[OFF_W2 + r * H + 2 * c + 1];
        W2s[r][c] = w;
    }
    for (int e = threadIdx.x; e < H; e += blockDim.x) {
        b1s[e] = float(ph[OFF_B1 + e]);
        b2s[e] = float(ph[OFF_B2 + e]);
        w3s[e] = float(ph[OFF_W3 + e]);
    }
    if (threadIdx.x == 0)
        b3s = float(ph[OFF_B3]);
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    half2v xh[F / 2];
#pragma unroll
    for (int c = 0; c < F / 2; ++c) {
        xh[c].x = _Float16(x[size_t(s) * F + 2 * c]);
        xh[c].y = _Float16(x[size_t(s) * F + 2 * c + 1]);
    }
    half2v h1[H / 2];
#pragma unroll
    for (int jj = 0; jj < H / 2; ++jj) {
        float a[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = 2 * jj + q;
            float acc = b1s[j];
#pragma unroll
            for (int c = 0; c < F / 2; ++c)
                acc = __builtin_amdgcn_fdot2(W1s[j][c], xh[c], acc, false);
            a[q] = acc > 0.0f ? acc : 0.0f;
        }
        h1[jj].x = _Float16(a[0]);
        h1[jj].y = _Float16(a[1]);
    }
    float yv = b3s;
    for (int j = 0; j < H; ++j) {
        float acc = b2s[j];
#pragma unroll
        for (int c = 0; c < H / 2; ++c)
            acc = __builtin_amdgcn_fdot2(W2s[j][c], h1[c], acc, false);
        yv += w3s[j] * (acc > 0.0f ? acc : 0.0f);
    }
    out[s] = yv;
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) for deterministic initialisation.
uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace
}  // namespace sv

using namespace sv;

struct sv_costmodel {
    float *d_p = nullptr, *d_m = nullptr, *d_v = nullptr;
    _Float16 *d_ph = nullptr;
    float *d_part = nullptr, *d_x = nullptr, *d_y = nullptr, *d_out = nullptr, *d_loss = nullptr;
    float *d_grad = nullptr;  // P floats
    size_t cap = 0;
    int t = 0;
    hipStream_t s = nullptr;
    bool half_fresh = false;
    uint64_t version = 1;  // changes whenever the parameters do
};

namespace {

#define CM_TRY(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                     \
            return SV_EDEVICE;                                                           \
        }                                                                                \
    } while (0)

int cm_reserve(sv_costmodel *m, size_t n)
{
    if (n <= m->cap)
        return SV_OK;
    CM_TRY(hipStreamSynchronize(m->s));
    if (m->d_x)
        (void)hipFree(m->d_x);
    if (m->d_y)
        (void)hipFree(m->d_y);
    if (m->d_out)
        (void)hipFree(m->d_out);
    m->d_x = m->d_y = m->d_out = nullptr;
    m->cap = 0;
    if (hipMalloc((void **)&m->d_x, n * F * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_y, n * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_out, n * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cost model: cannot allocate buffers for %zu samples", n);
        return SV_ENOMEM;
    }
    m->cap = n;
    return SV_OK;
}

int cm_refresh_half(sv_costmodel *m)
{
    if (m->half_fresh)
        return SV_OK;
    hipLaunchKernelGGL(k_mlp_to_half, dim3((P + 255) / 256), dim3(256), 0, m->s, m->d_p, m->d_ph);
    CM_TRY(hipGetLastError());
    m->half_fresh = true;
    return SV_OK;
}

int cm_check_data(const float *x, const float *y, int n, bool need_y)
{
    if (n < 1 || !x || (need_y && !y)) {
        set_error("cost model: bad data arguments");
        return SV_EINVAL;
    }
    for (size_t i = 0; i < size_t(n) * F; ++i)
        if (!std::isfinite(x[i])) {
            set_error("cost model: non-finite feature");
            return SV_EINVAL;
        }
    if (need_y)
        for (int i = 0; i < n; ++i)
            if (!std::isfinite(y[i])) {
                set_error("cost model: non-finite target");
                return SV_EINVAL;
            }
    return SV_OK;
}

// One forward/backward pass over the resident data; leaves partials in d_part.
int cm_grad_launch(sv_costmodel *m, int n, int &chunks)
{
    chunks = n < kMaxChunks ? n : kMaxChunks;
    hipLaunchKernelGGL(k_mlp_grad, dim3(chunks), dim3(H), 0, m->s, m->d_p, m->d_x, m->d_y, n, 2.0f / float(n),
                       m->d_part);
    CM_TRY(hipGetLastError());
    return SV_OK;
}

}  // namespace

namespace sv {

void sweep_features(int n, int dtype, const sv_sweep_record &r, float *f)
{
    static_assert(F == 16, "feature layout");
    const float fn = float(n);
    const bool pass = r.kind == SV_SWEEP_PASS;
    // tile bits among the top 8 index bits, and the contiguous low tile
    // bits (a pass tile reads runs of 2^that amplitudes)
    const uint64_t tm = pass ? r.tile_mask : 0;
    const int top = n > 8 ? __builtin_popcountll(tm >> (n - 8)) : __builtin_popcountll(tm);
    const int run = __builtin_ctzll(~tm);
    f[0] = float(r.k) / 8.0f;
    f[1] = float(r.c) / 8.0f;
    f[2] = std::log2(1.0f + float(r.num_gates)) / 8.0f;
    f[3] = float(r.lowest_target) / fn;
    f[4] = float(r.highest_target) / fn;
    f[5] = float(top) / 8.0f;
    f[6] = float(dtype);
    f[7] = pass ? 1.0f : 0.0f;
    f[8] = float(r.kind) / 7.0f;
    f[9] = float(std::log2(r.bytes > 1.0 ? r.bytes : 1.0)) / 40.0f;
    f[10] = float(r.blocks) / 8.0f;
    f[11] = float(r.term_blocks) / 8.0f;
    f[12] = float(r.variant_blocks) / 8.0f;
    f[13] = pass ? float(r.tile_log - pass_tile_log(dtype)) : 0.0f;
    f[14] = r.precision == SV_PREC_BF16X6 ? 1.0f : (r.precision == SV_PREC_BF16X3 ? 0.5f : 0.0f);
    f[15] = float(run) / 8.0f;
}

sv_sweep_record block_record(int n, int dtype, const Block &b, int precision)
{
    sv_sweep_record r{};
    r.k = b.k;
    r.c = b.c;
    r.lowest_target = *std::min_element(b.targets, b.targets + b.k);
    r.highest_target = *std::max_element(b.targets, b.targets + b.k);
    r.num_gates = b.ngates;
    r.bytes = block_bytes(n, dtype, b, b.targets, b.controls);
    r.flops = block_flops(n, b);
    r.kind = (b.k == 1 && b.diag) ? SV_SWEEP_DIAG1 : (b.k == 1) ? SV_SWEEP_GATE1
                                                                : dense_path(n, dtype, b.k, b.c, precision);
    return r;
}

// Physical bit of logical qubit q.
static inline int phys_of(const int *phys, int q)
{
    return phys ? phys[q] : q;
}

// The sweep a greedy group becomes (physical positions): its shape, padded to
// four targets where execution pads (the pad is the lowest free qubit >= 6).
static sv_sweep_record group_record(int n, int dtype, int precision, const std::vector<Block> &gates,
                                    const Group &g, const int *phys)
{
    Block b = group_shape(gates, g);
    if (b.k == 3 && pads_to_four(n, dtype, b.c, precision)) {
        uint64_t used = qubit_mask(b);
        int pick = -1;
        for (int q = 0; q < n && pick < 0; ++q)
            if (q >= 6 && !((used >> q) & 1))
                pick = q;
        for (int q = 0; q < n && pick < 0; ++q)
            if (!((used >> q) & 1))
                pick = q;
        b.targets[b.k++] = pick;
    }
    for (int j = 0; j < b.k; ++j)
        b.targets[j] = phys_of(phys, b.targets[j]);
    for (int j = 0; j < b.c; ++j)
        b.controls[j] = phys_of(phys, b.controls[j]);
    return block_record(n, dtype, b, precision);
}

sv_sweep_record pass_record(int n, int dtype, int precision, const PassGroup &w, const int *phys, int T)
{
    sv_sweep_record r{};
    r.kind = SV_SWEEP_PASS;
    uint64_t pm = 0, avoid = 0;
    for (int q = 0; q < n; ++q) {
        if ((w.qmask >> q) & 1)
            pm |= uint64_t(1) << phys_of(phys, q);
        if ((w.omask >> q) & 1)
            avoid |= uint64_t(1) << phys_of(phys, q);
    }
    r.k = __builtin_popcountll(pm);
    r.lowest_target = pm ? __builtin_ctzll(pm) : 0;
    r.highest_target = pm ? 63 - __builtin_clzll(pm) : 0;
    r.num_gates = w.ngates;
    const double amps = std::ldexp(1.0, n);
    const bool split = dtype == SV_C64 && precision == SV_PREC_BF16X6;
    r.bytes = 2.0 * (dtype == SV_C64 ? 8.0 : 16.0) * amps;
    r.blocks = int(w.subs.size());
    r.flops = double(r.blocks) * 126.0 * amps;
    r.mfma_flops = double(r.blocks) * (split ? 768.0 : 96.0) * amps;
    r.precision = split ? SV_PREC_BF16X6 : SV_PREC_NATIVE;
    for (size_t i = 0; i < w.subs.size(); ++i) {
        r.term_blocks += (!w.front[i].empty() || !w.back[i].empty()) ? 1 : 0;
        r.variant_blocks += w.vq[i] != 0 ? 1 : 0;
    }
    int tb[16];
    if (pass_tile_bits(n, T, pm, avoid, tb) == T) {
        r.tile_log = T;
        for (int b = 0; b < T; ++b)
            r.tile_mask |= uint64_t(1) << tb[b];
    }
    return r;
}

// Tile widths a kernel pass may take: the smallest, and twice it where the
// kernel has that form (not the complex64 split-BF16 kernel) and the state
// holds enough tiles of it.
static int pass_tile_options(int n, int dtype, int precision, int *opts)
{
    const int T0 = pass_tile_log(dtype);
    int k = 0;
    opts[k++] = T0;
    const bool split = dtype == SV_C64 && precision == SV_PREC_BF16X6;
    if (!split && n >= T0 + 1 + 6)
        opts[k++] = T0 + 1;
    return k;
}

// Feature rows of candidate sweeps and the predicted time of each (ms).
struct Ranker {
    int n, dtype;
    std::vector<float> feats;
    std::vector<double> gbytes;
    std::vector<double> ms;
    int add(const sv_sweep_record &r)
    {
        float f[F];
        sweep_features(n, dtype, r, f);
        feats.insert(feats.end(), f, f + F);
        gbytes.push_back(r.bytes * 1e-9);
        return int(gbytes.size()) - 1;
    }
    int run(sv_costmodel *m)
    {
        const int rows = int(gbytes.size());
        ms.assign(size_t(rows), 0.0);
        if (rows == 0)
            return SV_OK;
        std::vector<float> pred(static_cast<size_t>(rows));
        int rc = sv_costmodel_predict(m, feats.data(), rows, pred.data());
        if (rc != SV_OK)
            return rc;
        for (int i = 0; i < rows; ++i)
            ms[size_t(i)] = std::exp(double(pred[size_t(i)])) * gbytes[size_t(i)];
        return SV_OK;
    }
};

// Rows of one candidate pass plan: per kernel pass one row per tile option,
// per fallback pass its sweeps.
struct PlanRows {
    std::vector<std::vector<int>> pass_rows;  // rows of pass i (tile options, or its sweeps)
    std::vector<std::vector<int>> tiles;      // kernel pass i: the tile width of each row
};

static PlanRows plan_rows(Ranker &rk, int precision, const std::vector<Block> &gates,
                          const std::vector<PassGroup> &plan, const int *phys)
{
    PlanRows pr;
    int opts[2];
    const int nopt = pass_tile_options(rk.n, rk.dtype, precision, opts);
    for (const PassGroup &w : plan) {
        std::vector<int> rows, tiles;
        if (w.kernel) {
            for (int o = 0; o < nopt; ++o) {
                const sv_sweep_record r = pass_record(rk.n, rk.dtype, precision, w, phys, opts[o]);
                if (r.tile_log == 0)
                    continue;  // the pass does not fit this tile
                rows.push_back(rk.add(r));
                tiles.push_back(opts[o]);
            }
        } else {
            for (const Group &g : w.subs)
                rows.push_back(rk.add(group_record(rk.n, rk.dtype, precision, gates, g, phys)));
        }
        pr.pass_rows.push_back(std::move(rows));
        pr.tiles.push_back(std::move(tiles));
    }
    return pr;
}

// Predicted time of a plan with each kernel pass at its fastest tile (and
// those tiles written into the plan).
static double plan_time(const Ranker &rk, const PlanRows &pr, std::vector<PassGroup> *plan)
{
    double t = 0.0;
    for (size_t i = 0; i < pr.pass_rows.size(); ++i) {
        const std::vector<int> &rows = pr.pass_rows[i];
        if (pr.tiles[i].empty()) {
            for (int r : rows)
                t += rk.ms[size_t(r)];
            if (rows.empty() && plan && (*plan)[i].kernel)
                return HUGE_VAL;  // a kernel pass that fits no tile
            continue;
        }
        size_t best = 0;
        for (size_t o = 1; o < rows.size(); ++o)
            if (rk.ms[size_t(rows[o])] < rk.ms[size_t(rows[best])])
                best = o;
        t += rk.ms[size_t(rows[best])];
        if (plan)
            (*plan)[i].tile_log = pr.tiles[i][best];
    }
    return t;
}

int learned_pass_plan(sv_costmodel *m, int n, int dtype, int precision, const std::vector<Block> &gates,
                      int max_fused, const int *phys, int orders, std::vector<PassGroup> &plan, double *pred_ms)
{
    const int T0 = pass_tile_log(dtype);
    std::vector<std::vector<PassGroup>> cands;
    for (int pq = 6; pq <= kMaxPassQubits; ++pq)
        for (std::vector<PassGroup> &c : pass_plan_candidates(gates, pq, max_fused, n, T0, phys, orders))
            cands.push_back(std::move(c));
    Ranker rk{n, dtype, {}, {}, {}};
    std::vector<PlanRows> rows;
    rows.reserve(cands.size());
    for (const std::vector<PassGroup> &c : cands)
        rows.push_back(plan_rows(rk, precision, gates, c, phys));
    int rc = rk.run(m);
    if (rc != SV_OK)
        return rc;
    size_t best = 0;
    double tbest = HUGE_VAL;
    for (size_t i = 0; i < cands.size(); ++i) {
        const double t = plan_time(rk, rows[i], nullptr);
        if (t < tbest) {
            tbest = t;
            best = i;
        }
    }
    if (!std::isfinite(tbest)) {
        set_error("cost model: no finite prediction for any pass plan");
        return SV_EINVAL;
    }
    plan = std::move(cands[best]);
    plan_time(rk, rows[best], &plan);
    if (pred_ms)
        *pred_ms = tbest;
    return SV_OK;
}

int rank_plans(sv_costmodel *m, int n, int dtype, const std::vector<Block> &gates, int max_fused, int precision,
               int &chosen, float *pred_ms, const int *phys, std::vector<PassGroup> *pass_plan_out)
{
    chosen = max_fused;
    if (!m)
        return SV_OK;
    // greedy widths 1..max_fused
    Ranker rk{n, dtype, {}, {}, {}};
    std::vector<std::vector<int>> width_rows(size_t(max_fused) + 1);
    for (int k = 1; k <= max_fused; ++k)
        for (const Group &g : group_greedy(gates, k))
            width_rows[size_t(k)].push_back(rk.add(group_record(n, dtype, precision, gates, g, phys)));
    int rc = rk.run(m);
    if (rc != SV_OK)
        return rc;
    std::vector<double> tot(size_t(max_fused) + 1, 0.0);
    for (int k = 1; k <= max_fused; ++k)
        for (int r : width_rows[size_t(k)])
            tot[size_t(k)] += rk.ms[size_t(r)];
    // the LDS pass plans, on the gate list with diagonal pairs fused
    std::vector<PassGroup> pplan;
    double tp = HUGE_VAL;
    const std::vector<Block> pgates = prefuse_diagonal_pairs(gates);
    constexpr int kLearnedOrders = 8;
    rc = learned_pass_plan(m, n, dtype, precision, pgates, max_fused, phys, kLearnedOrders, pplan, &tp);
    if (rc != SV_OK)
        return rc;
    tot[0] = tp;
    double best = 0.0;
    bool finite = true, any = false;
    for (int cand = 1; cand <= max_fused + 1; ++cand) {
        const int c = cand == max_fused + 1 ? 0 : cand;  // widths first, then the pass plan
        if (pred_ms)
            pred_ms[cand - 1] = float(tot[size_t(c)]);
        if (!std::isfinite(tot[size_t(c)]))
            finite = false;
        if (!any || tot[size_t(c)] < best) {
            best = tot[size_t(c)];
            chosen = c;
            any = true;
        }
    }
    if (!finite)
        chosen = max_fused;
    if (pass_plan_out)
        *pass_plan_out = std::move(pplan);
    return SV_OK;
}

uint64_t costmodel_version(const sv_costmodel *m)
{
    return m ? m->version : 0;
}

}  // namespace sv

extern "C" {

int sv_costmodel_num_params(int *count)
{
    if (!count) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    *count = P;
    return SV_OK;
}

int sv_costmodel_create(uint64_t seed, sv_costmodel_handle *out)
{
    clear_error();
    if (!out) {
        set_error("NULL output");
        return SV_EINVAL;
    }
    sv_costmodel *m = new (std::nothrow) sv_costmodel();
    if (!m) {
        set_error("out of host memory");
        return SV_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&m->d_p, P * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_m, P * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_v, P * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_ph, P * sizeof(_Float16)) != hipSuccess ||
        hipMalloc((void **)&m->d_part, size_t(kMaxChunks) * PS * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_loss, sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->d_grad, P * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        sv_costmodel_destroy(m);
        set_error("cost model: device allocation failed");
        return SV_ENOMEM;
    }
    // He-uniform weights, zero biases
    std::vector<float> p(P, 0.0f);
    uint64_t st = seed;
    auto uni = [&]() { return double(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0); };
    const double a1 = std::sqrt(6.0 / F), a2 = std::sqrt(6.0 / H);
    for (int i = 0; i < H * F; ++i)
        p[OFF_W1 + i] = float((2.0 * uni() - 1.0) * a1);
    for (int i = 0; i < H * H; ++i)
        p[OFF_W2 + i] = float((2.0 * uni() - 1.0) * a2);
    for (int i = 0; i < H; ++i)
        p[OFF_W3 + i] = float((2.0 * uni() - 1.0) * a2);
    std::vector<float> z(P, 0.0f);
    if (hipMemcpy(m->d_p, p.data(), P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_m, z.data(), P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_v, z.data(), P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        sv_costmodel_destroy(m);
        set_error("cost model: upload failed");
        return SV_EDEVICE;
    }
    *out = m;
    return SV_OK;
}

int sv_costmodel_get_params(sv_costmodel_handle m, float *out)
{
    if (!m || !out) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    CM_TRY(hipStreamSynchronize(m->s));
    CM_TRY(hipMemcpy(out, m->d_p, P * sizeof(float), hipMemcpyDeviceToHost));
    return SV_OK;
}

int sv_costmodel_set_params(sv_costmodel_handle m, const float *in)
{
    if (!m || !in) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    for (int i = 0; i < P; ++i)
        if (!std::isfinite(in[i])) {
            set_error("cost model: non-finite parameter");
            return SV_EINVAL;
        }
    CM_TRY(hipStreamSynchronize(m->s));
    CM_TRY(hipMemcpy(m->d_p, in, P * sizeof(float), hipMemcpyHostToDevice));
    m->half_fresh = false;
    m->version += 1;
    return SV_OK;
}

int sv_costmodel_grad(sv_costmodel_handle m, const float *x, const float *y, int n, float *grad, float *loss)
{
    clear_error();
    if (!m || !grad) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    int rc = cm_check_data(x, y, n, true);
    if (rc != SV_OK || (rc = cm_reserve(m, size_t(n))) != SV_OK)
        return rc;
    CM_TRY(hipMemcpyAsync(m->d_x, x, size_t(n) * F * sizeof(float), hipMemcpyHostToDevice, m->s));
    CM_TRY(hipMemcpyAsync(m->d_y, y, size_t(n) * sizeof(float), hipMemcpyHostToDevice, m->s));
    int chunks = 0;
    if ((rc = cm_grad_launch(m, n, chunks)) != SV_OK)
        return rc;
    hipLaunchKernelGGL(k_mlp_update, dim3((P + 1 + 255) / 256), dim3(256), 0, m->s, m->d_p, m->d_m, m->d_v, m->d_part,
                       chunks, 0, 0.0f, 1.0f, 1.0f, 1.0f / float(n), m->d_grad, m->d_loss);
    CM_TRY(hipGetLastError());
    CM_TRY(hipMemcpyAsync(grad, m->d_grad, P * sizeof(float), hipMemcpyDeviceToHost, m->s));
    float l = 0.0f;
    CM_TRY(hipMemcpyAsync(&l, m->d_loss, sizeof(float), hipMemcpyDeviceToHost, m->s));
    CM_TRY(hipStreamSynchronize(m->s));
    if (loss)
        *loss = l;
    return SV_OK;
}

int sv_costmodel_train(sv_costmodel_handle m, const float *x, const float *y, int n, int epochs, float lr,
                       float *final_loss)
{
    clear_error();
    if (!m || epochs < 1 || !(lr > 0.0f) || !std::isfinite(lr)) {
        set_error("cost model: bad training arguments");
        return SV_EINVAL;
    }
    int rc = cm_check_data(x, y, n, true);
    if (rc != SV_OK || (rc = cm_reserve(m, size_t(n))) != SV_OK)
        return rc;
    CM_TRY(hipMemcpyAsync(m->d_x, x, size_t(n) * F * sizeof(float), hipMemcpyHostToDevice, m->s));
    CM_TRY(hipMemcpyAsync(m->d_y, y, size_t(n) * sizeof(float), hipMemcpyHostToDevice, m->s));
    for (int e = 0; e < epochs; ++e) {
        int chunks = 0;
        if ((rc = cm_grad_launch(m, n, chunks)) != SV_OK)
            return rc;
        m->t += 1;
        const float c1 = float(1.0 - std::pow(0.9, m->t)), c2 = float(1.0 - std::pow(0.999, m->t));
        hipLaunchKernelGGL(k_mlp_update, dim3((P + 1 + 255) / 256), dim3(256), 0, m->s, m->d_p, m->d_m, m->d_v,
                           m->d_part, chunks, 1, lr, c1, c2, 1.0f / float(n), m->d_grad, m->d_loss);
        CM_TRY(hipGetLastError());
    }
    m->half_fresh = false;
    m->version += 1;
    float l = 0.0f;
    CM_TRY(hipMemcpyAsync(&l, m->d_loss, sizeof(float), hipMemcpyDeviceToHost, m->s));
    CM_TRY(hipStreamSynchronize(m->s));
    if (final_loss)
        *final_loss = l;
    return SV_OK;
}

int sv_costmodel_predict(sv_costmodel_handle m, const float *x, int n, float *out)
{
    if (!m || !out) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    int rc = cm_check_data(x, nullptr, n, false);
    if (rc != SV_OK || (rc = cm_reserve(m, size_t(n))) != SV_OK || (rc = cm_refresh_half(m)) != SV_OK)
        return rc;
    CM_TRY(hipMemcpyAsync(m->d_x, x, size_t(n) * F * sizeof(float), hipMemcpyHostToDevice, m->s));
    hipLaunchKernelGGL(k_mlp_predict, dim3((n + 255) / 256), dim3(256), 0, m->s, m->d_ph, m->d_x, n, m->d_out);
    CM_TRY(hipGetLastError());
    CM_TRY(hipMemcpyAsync(out, m->d_out, size_t(n) * sizeof(float), hipMemcpyDeviceToHost, m->s));
    CM_TRY(hipStreamSynchronize(m->s));
    return SV_OK;
}

int sv_costmodel_destroy(sv_costmodel_handle m)
{
    if (!m)
        return SV_OK;
    if (m->s)
        (void)hipStreamSynchronize(m->s);
    float *bufs[] = {m->d_p, m->d_m, m->d_v, m->d_part, m->d_x, m->d_y, m->d_out, m->d_loss, m->d_grad};
    for (float *b : bufs)
        if (b)
            (void)hipFree(b);
    if (m->d_ph)
        (void)hipFree(m->d_ph);
    if (m->s)
        (void)hipStreamDestroy(m->s);
    delete m;
    return SV_OK;
}

int sv_sweep_features(int n, int dtype, const sv_sweep_record *recs, int count, float *out)
{
    if (n < 1 || n > SV_MAX_QUBITS || (dtype != SV_C64 && dtype != SV_C128) || count < 0 ||
        (count > 0 && (!recs || !out))) {
        set_error("sv_sweep_features: bad arguments");
        return SV_EINVAL;
    }
    for (int i = 0; i < count; ++i)
        sweep_features(n, dtype, recs[i], out + size_t(i) * F);
    return SV_OK;
}

int sv_sweep_targets(const sv_sweep_record *recs, int count, float *out)
{
    if (count < 0 || (count > 0 && (!recs || !out))) {
        set_error("sv_sweep_targets: bad arguments");
        return SV_EINVAL;
    }
    for (int i = 0; i < count; ++i) {
        const double ms = recs[i].ms > 1e-6f ? double(recs[i].ms) : 1e-6;
        const double gb = recs[i].bytes > 1.0 ? recs[i].bytes * 1e-9 : 1e-9;
        out[i] = float(std::log(ms / gb));
    }
    return SV_OK;
}

int sv_costmodel_rank(sv_costmodel_handle m, int n, int dtype, const sv_gate *gates, int ngates, int max_fused,
                      int *chosen, float *predicted_ms)
{
    clear_error();
    if (!m || !chosen || max_fused < 1 || max_fused > SV_MAX_TARGETS) {
        set_error("sv_costmodel_rank: bad arguments");
        return SV_EINVAL;
    }
    uint64_t bytes;
    int rc = sv_state_bytes(n, dtype, &bytes);
    if (rc != SV_OK)
        return rc;
    std::vector<Block> blocks;
    sv_plan_opts o{SV_PLAN_PLAIN, max_fused, SV_PREC_NATIVE, 0, 0, 0};
    if ((rc = plan_circuit(n, dtype, gates, ngates, o, blocks)) != SV_OK)
        return rc;
    return rank_plans(m, n, dtype, blocks, max_fused, dtype == SV_C64 ? SV_PREC_BF16X6 : SV_PREC_NATIVE, *chosen,
                      predicted_ms, nullptr, nullptr);
}

}  // extern "C"
