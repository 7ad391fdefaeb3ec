// The extern "C" entry points declared in include/sv.h.
//
// Every entry point validates its arguments on the host first (so argument
// errors are reported without touching the GPU), then queues kernels on the
// handle's stream.  Gate application returns without waiting; read-outs
// synchronise and copy their (small) results to host memory.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sv_internal.h"

namespace sv {

static thread_local std::string g_error;

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
}

void clear_error()
{
    g_error.clear();
}

}  // namespace sv

using namespace sv;

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                     \
            return SV_EDEVICE;                                                           \
        }                                                                                \
    } while (0)

// A plan kept on a handle for a circuit structure: the key lists the
// options, the state's qubit map and, per gate, its width, controls, qubits,
// diagonality and whether it is a pure phase (everything the planners read).
struct PlanCacheEntry {
    std::vector<uint64_t> key;
    int width = 0;                     // SV_PLAN_LEARNED: greedy width chosen, 0 = the pass plan
    std::vector<sv::PassGroup> plan;   // pass plan on the gate list with diagonal pairs pre-fused
};

struct sv_state {
    int n = 0;
    int dtype = 0;
    uint64_t bytes = 0;
    void *d_state = nullptr;
    bool owned = false;
    int device = 0;
    hipStream_t stream = nullptr;
    int qmap[SV_MAX_QUBITS] = {};
    // device scratch for read-outs
    double *d_scratch = nullptr;
    uint64_t scratch_bytes = 0;
    // pinned host staging
    void *h_pinned = nullptr;
    uint64_t pinned_bytes = 0;
    // device arena holding block matrices of the current circuit, and its
    // pinned host staging (reused once the previous upload has completed)
    void *d_arena = nullptr;
    uint64_t arena_bytes = 0;
    void *h_arena = nullptr;
    uint64_t h_arena_bytes = 0;
    hipEvent_t arena_done = nullptr;
    bool arena_pending = false;
    // plans of recent circuit structures, most recent first
    std::vector<PlanCacheEntry> plan_cache;
    // sweep timing
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Pending {
        sv_sweep_record rec;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    // cost model consulted by SV_PLAN_LEARNED (not owned)
    sv_costmodel *model = nullptr;
};

struct sv_plan {
    int n = 0;
    int dtype = 0;
    int precision = 0;
    int ngates = 0;
    std::vector<Block> blocks;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard()
    {
        if (changed)
            (void)hipSetDevice(prev);
    }
};

uint64_t amp_bytes(int dtype)
{
    return dtype == SV_C64 ? 8 : 16;
}

bool identity_map(const sv_state *h)
{
    for (int q = 0; q < h->n; ++q)
        if (h->qmap[q] != q)
            return false;
    return true;
}

int check_handle(sv_handle h)
{
    if (h == nullptr) {
        set_error("NULL handle");
        return SV_EINVAL;
    }
    return SV_OK;
}

int ensure_scratch(sv_state *h, uint64_t bytes)
{
    if (bytes <= h->scratch_bytes)
        return SV_OK;
    if (h->d_scratch) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(hipFree(h->d_scratch));
        h->d_scratch = nullptr;
        h->scratch_bytes = 0;
    }
    uint64_t want = std::max<uint64_t>(bytes, uint64_t(1) << 20);
    if (hipMalloc((void **)&h->d_scratch, want) != hipSuccess) {
        (void)hipGetLastError();
        h->d_scratch = nullptr;
        set_error("cannot allocate %llu bytes of device scratch", (unsigned long long)want);
        return SV_ENOMEM;
    }
    h->scratch_bytes = want;
    return SV_OK;
}

int ensure_pinned(sv_state *h, uint64_t bytes)
{
    if (bytes <= h->pinned_bytes)
        return SV_OK;
    if (h->h_pinned) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(hipHostFree(h->h_pinned));
        h->h_pinned = nullptr;
        h->pinned_bytes = 0;
    }
    uint64_t want = std::max<uint64_t>(bytes, uint64_t(1) << 20);
    if (hipHostMalloc(&h->h_pinned, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        h->h_pinned = nullptr;
        set_error("cannot allocate %llu bytes of pinned host memory", (unsigned long long)want);
        return SV_ENOMEM;
    }
    h->pinned_bytes = want;
    return SV_OK;
}

// Device bytes of a block's matrix in the state's precision (256-aligned),
// 0 for one-target blocks (their 2x2 matrix travels as kernel arguments).
uint64_t matrix_bytes(const sv_state *h, int k)
{
    if (k < 2)
        return 0;
    const uint64_t d = uint64_t(1) << k;
    return (d * d * amp_bytes(h->dtype) + 255) & ~uint64_t(255);
}

// Make the pinned staging buffer and the device arena hold `total` bytes; the
// staging buffer is free to overwrite on return (the previous call's uploads
// have been read).
int ensure_arena(sv_state *h, uint64_t total)
{
    if (h->arena_pending) {
        HIP_TRY(hipEventSynchronize(h->arena_done));
        h->arena_pending = false;
    }
    if (total == 0)
        return SV_OK;
    if (total > h->h_arena_bytes) {
        if (h->h_arena)
            HIP_TRY(hipHostFree(h->h_arena));
        h->h_arena = nullptr;
        h->h_arena_bytes = 0;
        if (hipHostMalloc(&h->h_arena, total, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot allocate %llu bytes of pinned matrix staging", (unsigned long long)total);
            return SV_ENOMEM;
        }
        h->h_arena_bytes = total;
    }
    if (total > h->arena_bytes) {
        if (h->d_arena) {
            HIP_TRY(hipStreamSynchronize(h->stream));
            HIP_TRY(hipFree(h->d_arena));
        }
        h->d_arena = nullptr;
        h->arena_bytes = 0;
        if (hipMalloc(&h->d_arena, total) != hipSuccess) {
            (void)hipGetLastError();
            set_error("cannot allocate %llu bytes of device matrix arena", (unsigned long long)total);
            return SV_ENOMEM;
        }
        h->arena_bytes = total;
    }
    return SV_OK;
}

// Write block b's matrix into the staging buffer at byte offset off.
void stage_matrix(sv_state *h, const Block &b, uint64_t off)
{
    char *stage = static_cast<char *>(h->h_arena) + off;
    const size_t dd = size_t(1) << (2 * b.k);
    if (h->dtype == SV_C64) {
        float *dst = reinterpret_cast<float *>(stage);
        for (size_t j = 0; j < dd; ++j) {
            dst[2 * j] = float(b.U[j].real());
            dst[2 * j + 1] = float(b.U[j].imag());
        }
    } else {
        double *dst = reinterpret_cast<double *>(stage);
        for (size_t j = 0; j < dd; ++j) {
            dst[2 * j] = b.U[j].real();
            dst[2 * j + 1] = b.U[j].imag();
        }
    }
}

// Queue the copy of staging bytes [lo, hi) to the device arena.
int upload_range(sv_state *h, uint64_t lo, uint64_t hi)
{
    if (hi <= lo)
        return SV_OK;
    HIP_TRY(hipMemcpyAsync(static_cast<char *>(h->d_arena) + lo, static_cast<const char *>(h->h_arena) + lo, hi - lo,
                           hipMemcpyHostToDevice, h->stream));
    return SV_OK;
}

int take_event(sv_state *h, hipEvent_t &ev)
{
    if (h->ev_used == h->ev_pool.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        h->ev_pool.push_back(e);
    }
    ev = h->ev_pool[h->ev_used++];
    return SV_OK;
}

// Open a timed sweep: record the start event (no-op unless profiling).
int prof_begin(sv_state *h, sv_state::Pending &p)
{
    if (!h->profiling)
        return SV_OK;
    int rc = take_event(h, p.a);
    if (rc == SV_OK)
        rc = take_event(h, p.b);
    if (rc != SV_OK)
        return rc;
    HIP_TRY(hipEventRecord(p.a, h->stream));
    return SV_OK;
}

int prof_end(sv_state *h, sv_state::Pending &p)
{
    if (!h->profiling)
        return SV_OK;
    HIP_TRY(hipEventRecord(p.b, h->stream));
    h->pending.push_back(p);
    return SV_OK;
}

// A dense 3-target block runs faster on the matrix cores as a 4-target one:
// U (x) I on one extra free qubit (the lowest free physical bit >= 6, else the
// lowest free one).
Block pad_to_four(const sv_state *h, const Block &b)
{
    uint64_t used = 0;
    for (int j = 0; j < b.k; ++j)
        used |= uint64_t(1) << b.targets[j];
    for (int j = 0; j < b.c; ++j)
        used |= uint64_t(1) << b.controls[j];
    int pick = -1, pick_any = -1;
    for (int q = 0; q < h->n; ++q) {
        if ((used >> q) & 1)
            continue;
        const int p = h->qmap[q];
        if (pick_any < 0 || p < h->qmap[pick_any])
            pick_any = q;
        if (p >= 6 && (pick < 0 || p < h->qmap[pick]))
            pick = q;
    }
    if (pick < 0)
        pick = pick_any;
    Block o = b;
    o.k = 4;
    o.targets[3] = pick;
    o.U.assign(256, cd(0.0, 0.0));
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c)
            if ((r >> 3) == (c >> 3))
                o.U[size_t(r) * 16 + c] = b.U[size_t(r & 7) * 8 + (c & 7)];
    return o;
}

bool padded_exec(const sv_state *h, const Block &b, int precision)
{
    return b.k == 3 && pads_to_four(h->n, h->dtype, b.c, precision);
}

// Launch one block's sweep (its matrix, if any, already at dU on the device)
// and account for it.
int launch_block(sv_state *h, const Block &b, const void *dU, int precision, size_t index, sv_run_stats &acc)
{
    int pt[SV_MAX_TARGETS], pc[SV_MAX_CONTROLS];
    for (int j = 0; j < b.k; ++j)
        pt[j] = h->qmap[b.targets[j]];
    for (int j = 0; j < b.c; ++j)
        pc[j] = h->qmap[b.controls[j]];
    sv_state::Pending pr{};
    pr.rec.k = b.k;
    pr.rec.c = b.c;
    pr.rec.lowest_target = *std::min_element(pt, pt + b.k);
    pr.rec.highest_target = *std::max_element(pt, pt + b.k);
    pr.rec.num_gates = b.ngates;
    pr.rec.bytes = block_bytes(h->n, h->dtype, b, pt, pc);
    pr.rec.flops = block_flops(h->n, b);
    pr.rec.kind = (b.k == 1 && b.diag) ? SV_SWEEP_DIAG1
                  : (b.k == 1)         ? SV_SWEEP_GATE1
                                       : dense_path(h->n, h->dtype, b.k, b.c, precision);
    int rc = prof_begin(h, pr);
    if (rc != SV_OK)
        return rc;
    hipError_t e;
    if (b.k == 1 && b.diag) {
        e = launch_diag1(h->d_state, h->n, h->dtype, b.U[0], b.U[3], pt[0], pc, b.c, h->stream);
    } else if (b.k == 1) {
        cd u[4] = {b.U[0], b.U[1], b.U[2], b.U[3]};
        e = launch_gate1(h->d_state, h->n, h->dtype, u, pt[0], pc, b.c, h->stream);
    } else {
        e = launch_gatek(h->d_state, h->n, h->dtype, dU, b.k, pt, pc, b.c, precision, h->stream);
    }
    if (e != hipSuccess) {
        set_error("gate sweep %zu launch failed: %s", index, hipGetErrorString(e));
        return SV_EDEVICE;
    }
    rc = prof_end(h, pr);
    if (rc != SV_OK)
        return rc;
    acc.sweeps += 1;
    if (b.ngates > 1)
        acc.fused_blocks += 1;
    acc.algorithmic_bytes += pr.rec.bytes;
    acc.flops += pr.rec.flops;
    return SV_OK;
}

// Run already formed blocks: all matrices in one upload, then every sweep.
int run_blocks(sv_state *h, const std::vector<Block> &blocks_in, int precision, int ngates, sv_run_stats *st)
{
    std::vector<Block> blocks;
    blocks.reserve(blocks_in.size());
    std::vector<uint64_t> offs(blocks_in.size(), 0);
    uint64_t total = 0;
    for (size_t i = 0; i < blocks_in.size(); ++i) {
        blocks.push_back(padded_exec(h, blocks_in[i], precision) ? pad_to_four(h, blocks_in[i]) : blocks_in[i]);
        offs[i] = total;
        total += matrix_bytes(h, blocks.back().k);
    }
    int rc = ensure_arena(h, total);
    if (rc != SV_OK)
        return rc;
    for (size_t i = 0; i < blocks.size(); ++i)
        if (blocks[i].k >= 2)
            stage_matrix(h, blocks[i], offs[i]);
    rc = upload_range(h, 0, total);
    if (rc != SV_OK)
        return rc;
    sv_run_stats acc{};
    acc.gates = ngates;
    for (size_t i = 0; i < blocks.size() && rc == SV_OK; ++i)
        rc = launch_block(h, blocks[i], static_cast<const char *>(h->d_arena) + offs[i], precision, i, acc);
    if (total > 0) {
        HIP_TRY(hipEventRecord(h->arena_done, h->stream));
        h->arena_pending = true;
    }
    if (rc == SV_OK && st)
        *st = acc;
    return rc;
}

// Run a grouped circuit: the blocks are formed, uploaded and launched in
// chunks of 1, 2, 4, ... blocks, so the host fuses the later blocks while the
// GPU is already sweeping the earlier ones.  Chunk c's matrices go up in one
// copy queued before chunk c's sweeps (all on the handle's stream).
int run_groups(sv_state *h, const std::vector<Block> &gates, const std::vector<Group> &groups, int precision,
               int ngates, sv_run_stats *st)
{
    const size_t nb = groups.size();
    std::vector<uint64_t> offs(nb, 0);
    uint64_t total = 0;
    for (size_t i = 0; i < nb; ++i) {
        const Group &g = groups[i];
        const Block &first = gates[size_t(g.members[0])];
        const int k = g.members.size() == 1 ? first.k : __builtin_popcountll(g.qmask);
        const int c = g.members.size() == 1 ? first.c : 0;
        const bool pad = k == 3 && pads_to_four(h->n, h->dtype, c, precision);
        offs[i] = total;
        total += matrix_bytes(h, pad ? 4 : k);
    }
    int rc = ensure_arena(h, total);
    if (rc != SV_OK)
        return rc;
    sv_run_stats acc{};
    acc.gates = ngates;
    std::vector<const Block *> mem;
    std::vector<Block> chunk;
    for (size_t next = 0, size = 1; next < nb && rc == SV_OK; next += size, size *= 2) {
        const size_t end = std::min(nb, next + size);
        chunk.clear();
        for (size_t i = next; i < end; ++i) {
            mem.clear();
            for (int m : groups[i].members)
                mem.push_back(&gates[size_t(m)]);
            Block b = fuse(mem, groups[i].qmask);
            if (padded_exec(h, b, precision))
                b = pad_to_four(h, b);
            if (b.k >= 2)
                stage_matrix(h, b, offs[i]);
            chunk.push_back(std::move(b));
        }
        const uint64_t hi = end < nb ? offs[end] : total;
        rc = upload_range(h, offs[next], hi);
        for (size_t i = next; i < end && rc == SV_OK; ++i)
            rc = launch_block(h, chunk[i - next], static_cast<const char *>(h->d_arena) + offs[i], precision, i, acc);
    }
    if (total > 0) {
        HIP_TRY(hipEventRecord(h->arena_done, h->stream));
        h->arena_pending = true;
    }
    if (rc == SV_OK && st)
        *st = acc;
    return rc;
}

// One pass of an SV_PLAN_PASSES plan: its gates grouped into sub-blocks of at
// most four qubits (pass kernel; phase gates reaching outside the tile ride on
// them as per-tile phases) or, when some gate is wider or the state is below
// the pass tile, into ordinary <= max_fused sweeps.
struct PassWork : PassGroup {
    uint64_t off = 0;        // arena range of the pass: [off, off + bytes)
    uint64_t bytes = 0;
    uint64_t nterm_max = 0;  // bound on the pass's phase terms
    bool split = false;      // complex64 blocks as split BF16 products (SV_PREC_BF16X6)
    bool presplit = false;   // split, no phase terms: matrices staged split (pass_presplit)
};

// Monomials of a phase gate's angle: a diagonal gate on qubits Q (targets,
// then controls) multiplies basis state x by exp(i f(x)), f(x) = arg U[x_t]
// when every control bit is 1, else 0.  Written as a sum over subsets S of Q,
// f(x) = sum_S alpha_S prod_{q in S} x_q, alpha_S = sum_{T subset of S}
// (-1)^{|S \ T|} f(T) (Moebius inversion over the subset lattice).
static void phase_monomials(const Block &g, int qubits[kMaxPhaseQubits], int &nq, std::vector<double> &alpha)
{
    nq = 0;
    for (int j = 0; j < g.k; ++j)
        qubits[nq++] = g.targets[j];
    for (int j = 0; j < g.c; ++j)
        qubits[nq++] = g.controls[j];
    const int N = 1 << nq, dk = 1 << g.k, cm = ((1 << g.c) - 1) << g.k;
    alpha.assign(size_t(N), 0.0);
    for (int x = 0; x < N; ++x)
        if ((x & cm) == cm) {
            const cd u = g.U[size_t(x & (dk - 1)) * dk + (x & (dk - 1))];
            alpha[size_t(x)] = std::atan2(u.imag(), u.real());
        }
    for (int b = 0; b < nq; ++b)
        for (int x = 0; x < N; ++x)
            if ((x >> b) & 1)
                alpha[size_t(x)] -= alpha[size_t(x ^ (1 << b))];
}

// A gate with its qubits outside the tile fixed: `ones` holds the logical
// qubits (among those outside tmask) whose index bit is 1.  A phase gate
// (diagonal, <= kMaxPhaseQubits qubits) becomes the diagonal block on its
// in-tile qubits (with none left, k = 0 and U[0] is the scalar phase); any
// other gate has only controls outside, and
// becomes itself on its in-tile controls where those outer controls are all 1,
// else the identity (k = 0, U[0] = 1).
static Block restrict_phase(const Block &g, uint64_t tmask, uint64_t ones)
{
    if (!is_phase_gate(g)) {
        Block o = g;
        o.c = 0;
        for (int j = 0; j < g.c; ++j) {
            const int q = g.controls[j];
            if ((tmask >> q) & 1) {
                o.controls[o.c++] = q;
            } else if (!((ones >> q) & 1)) {
                Block id;
                id.k = 0;
                id.U.assign(1, cd(1.0, 0.0));
                id.diag = true;
                id.ngates = g.ngates;
                return id;
            }
        }
        return o;
    }
    int qs[kMaxPhaseQubits + 1], nq = 0;
    for (int j = 0; j < g.k; ++j)
        qs[nq++] = g.targets[j];
    for (int j = 0; j < g.c; ++j)
        qs[nq++] = g.controls[j];
    Block o;
    int pos[kMaxPhaseQubits + 1];
    for (int j = 0; j < nq; ++j)
        if ((tmask >> qs[j]) & 1) {
            pos[j] = o.k;
            o.targets[o.k++] = qs[j];
        } else {
            pos[j] = -1;
        }
    const int d = 1 << o.k, dk = 1 << g.k, cm = ((1 << g.c) - 1) << g.k;
    o.U.assign(size_t(d) * d, cd(0.0, 0.0));
    for (int y = 0; y < d; ++y) {
        int x = 0;  // the gate's own index: targets, then controls
        for (int j = 0; j < nq; ++j) {
            const int bit = pos[j] >= 0 ? ((y >> pos[j]) & 1) : int((ones >> qs[j]) & 1);
            x |= bit << j;
        }
        o.U[size_t(y) * d + y] = (x & cm) == cm ? g.U[size_t(x & (dk - 1)) * dk + (x & (dk - 1))] : cd(1.0, 0.0);
    }
    o.diag = true;
    o.ngates = g.ngates;
    return o;
}

// Stage a kernel pass (descriptors, then the 16 x 16 matrices) and launch it.
int stage_launch_pass(sv_state *h, const std::vector<Block> &gates, const PassWork &w, bool launch, size_t index,
                      sv_run_stats &acc)
{
    uint64_t phys = 0;
    int lo = h->n, hi = -1;
    for (int q = 0; q < h->n; ++q)
        if ((w.qmask >> q) & 1) {
            const int p = h->qmap[q];
            phys |= uint64_t(1) << p;
            lo = std::min(lo, p);
            hi = std::max(hi, p);
        }
    uint64_t avoid = 0;  // outer qubits of the pass's phase gates stay outside the tile
    for (int q = 0; q < h->n; ++q)
        if ((w.omask >> q) & 1)
            avoid |= uint64_t(1) << h->qmap[q];
    int tb[16];
    const size_t nsub = w.subs.size();
    // the planner's tile width if it set one (the split kernel has the
    // smallest only), else by the pass's blocks; the smallest if the pass
    // does not fit the wider tile
    int T = -1;
    if (w.tile_log > 0 && !(w.split && w.tile_log != pass_tile_log(h->dtype)))
        T = pass_tile_bits(h->n, w.tile_log, phys, avoid, tb);
    if (T < 0)
        T = pass_tile_bits(h->n, pass_tile_log_for(h->n, h->dtype, int(nsub)), phys, avoid, tb);
    if (T < 0)
        T = pass_tile_bits(h->n, pass_tile_log(h->dtype), phys, avoid, tb);
    if (T < 0) {
        set_error("pass %zu does not fit the pass tile", index);
        return SV_EINVAL;
    }
    int slot_of[64];
    for (int b = 0; b < T; ++b)
        slot_of[tb[b]] = b;
    const uint64_t S = amp_bytes(h->dtype);
    const uint64_t mat16 = w.presplit ? kPresplitBytes : (256 * S + 255) & ~uint64_t(255);
    const uint64_t terms = w.off + ((nsub * sizeof(PassSub) + 255) & ~uint64_t(255));
    const uint64_t mats = terms + ((w.nterm_max * sizeof(PassTerm) + 255) & ~uint64_t(255));
    if (!launch) {
        PassSub *desc = reinterpret_cast<PassSub *>(static_cast<char *>(h->h_arena) + w.off);
        PassTerm *tt = reinterpret_cast<PassTerm *>(static_cast<char *>(h->h_arena) + terms);
        uint64_t nt = 0;
        std::vector<const Block *> mem;
        std::vector<double> alpha;
        uint64_t moff = mats;
        uint32_t pslot = 0;
        std::vector<Block> restricted;
        for (size_t i = 0; i < nsub; ++i) {
            const uint64_t vq = w.vq[i];
            const int nv = __builtin_popcountll(vq);
            int vql[kMaxVariantBits];
            for (int q = 0, j = 0; q < h->n; ++q)
                if ((vq >> q) & 1)
                    vql[j++] = q;
            // variant 0 (all variant qubits 0) fixes the slot layout
            auto build = [&](uint32_t var) {
                uint64_t ones = 0;
                for (int j = 0; j < nv; ++j)
                    if ((var >> j) & 1)
                        ones |= uint64_t(1) << vql[j];
                mem.clear();
                restricted.clear();
                restricted.reserve(w.subs[i].members.size());
                cd scalar(1.0, 0.0);
                for (int m : w.subs[i].members) {
                    const Block &g = gates[size_t(m)];
                    if ((qubit_mask(g) & ~w.qmask) == 0) {
                        mem.push_back(&g);
                        continue;
                    }
                    // a phase gate reaching outside the tile (variant blocks only)
                    restricted.push_back(restrict_phase(g, w.qmask, ones));
                    if (restricted.back().k == 0) {
                        scalar *= restricted.back().U[0];
                        restricted.pop_back();
                    } else {
                        mem.push_back(&restricted.back());
                    }
                }
                Block b;
                if (mem.empty() || nv > 0) {
                    b = fuse(mem, w.subs[i].qmask, true);
                } else {
                    b = densify(fuse(mem, w.subs[i].qmask));
                }
                for (cd &u : b.U)
                    u *= scalar;
                return b;
            };
            Block b = build(0);
            // slots: the block's qubits, then the in-tile qubits of its phase
            // gates, then the lowest free tile slots (identity on all of these)
            int slots[4], kk = 0;
            uint32_t used = 0;
            int lq_of_slot[4] = {-1, -1, -1, -1};
            for (int j = 0; j < b.k; ++j) {
                lq_of_slot[kk] = b.targets[j];
                slots[kk] = slot_of[h->qmap[b.targets[j]]];
                used |= 1u << slots[kk++];
            }
            for (int q = 0; q < h->n; ++q) {
                if (!((w.subs[i].qmask >> q) & 1))
                    continue;
                const int sl = slot_of[h->qmap[q]];
                if ((used >> sl) & 1)
                    continue;
                if (kk == 4) {
                    set_error("pass %zu: block %zu spans more than four tile slots", index, i);
                    return SV_EINVAL;
                }
                lq_of_slot[kk] = q;
                slots[kk++] = sl;
                used |= 1u << sl;
            }
            for (int sl = 0; kk < 4 && sl < T; ++sl)
                if (!((used >> sl) & 1)) {
                    slots[kk++] = sl;
                    used |= 1u << sl;
                }
            PassSub d{};
            for (int r = 0; r < 16; ++r)
                for (int j = 0; j < 4; ++j)
                    if ((r >> j) & 1)
                        d.xc[r] |= 1u << slots[j];
            int sorted[4] = {slots[0], slots[1], slots[2], slots[3]};
            std::sort(sorted, sorted + 4);
            for (int j = 0; j < 4; ++j)
                d.tslot_m[j] = (1u << sorted[j]) - 1u;
            d.u_off = moff;
            d.nvar = uint32_t(nv);
            for (int j = 0; j < nv; ++j)
                d.vpos[j] = uint8_t(h->qmap[vql[j]]);
            moff += (uint64_t(1) << nv) * mat16;
            // phase terms: (physical outer mask, block-local slot mask, side)
            d.t_off = terms + nt * sizeof(PassTerm);
            const uint64_t first = nt;
            // angle -> fixed-point turns (2^64 per turn); equal monomials merge
            auto add_term = [&](PassTerm t, double a) {
                double f = a / (2.0 * M_PI);
                f -= std::floor(f);
                t.turn = uint64_t(std::ldexp(f, 64) >= 18446744073709551615.0 ? 0.0 : std::ldexp(f, 64));
                for (uint64_t e = first; e < nt; ++e)
                    if (tt[e].omask == t.omask && tt[e].smask == t.smask && tt[e].back == t.back) {
                        tt[e].turn += t.turn;
                        return;
                    }
                if (nt < w.nterm_max)
                    tt[nt] = t;
                ++nt;
            };
            for (int side = 0; side < 2; ++side)
                for (int m : (side ? w.back[i] : w.front[i])) {
                    int qs[kMaxPhaseQubits], nq = 0;
                    phase_monomials(gates[size_t(m)], qs, nq, alpha);
                    for (int x = 1; x < (1 << nq); ++x) {
                        if (alpha[size_t(x)] == 0.0)
                            continue;
                        PassTerm t{};
                        for (int j = 0; j < nq; ++j) {
                            if (!((x >> j) & 1))
                                continue;
                            const int q = qs[j];
                            if ((w.omask >> q) & 1) {
                                t.omask |= uint64_t(1) << h->qmap[q];
                                continue;
                            }
                            int pos = -1;
                            for (int s2 = 0; s2 < 4; ++s2)
                                if (lq_of_slot[s2] == q)
                                    pos = s2;
                            if (pos < 0) {
                                set_error("pass %zu: phase gate %d outside block %zu", index, m, i);
                                return SV_EINVAL;
                            }
                            t.smask |= 1u << pos;
                        }
                        t.back = (side == 1 && t.smask != 0) ? 1u : 0u;
                        add_term(t, alpha[size_t(x)]);
                    }
                    // the constant monomial (x = 0) multiplies the whole tile
                    if (alpha[0] != 0.0)
                        add_term(PassTerm{}, alpha[0]);
                    if (nt > w.nterm_max) {
                        set_error("pass %zu: phase term table overflow", index);
                        return SV_EINVAL;
                    }
                }
            d.nterm = uint32_t(nt - first);
            if (d.nterm > 0) {
                if (pslot >= uint32_t(kMaxTermBlocks)) {
                    set_error("pass %zu: more than %d blocks with phase terms", index, kMaxTermBlocks);
                    return SV_EINVAL;
                }
                d.pslot = pslot++;
            }
            desc[i] = d;
            // U (x) I on the padding slots: row/column bits >= b.k must agree
            for (uint32_t var = 0; var < (1u << nv); ++var) {
                const Block bv = var == 0 ? b : build(var);
                Block u4;
                u4.k = 4;
                u4.U.assign(256, cd(0.0, 0.0));
                const int dk = 1 << bv.k;
                for (int r = 0; r < 16; ++r)
                    for (int c = 0; c < 16; ++c)
                        if ((r >> bv.k) == (c >> bv.k))
                            u4.U[size_t(r) * 16 + c] = bv.U[size_t(r & (dk - 1)) * dk + (c & (dk - 1))];
                if (w.presplit)
                    pass_presplit(u4.U.data(), static_cast<char *>(h->h_arena) + d.u_off + var * mat16);
                else
                    stage_matrix(h, u4, d.u_off + var * mat16);
            }
        }
        return SV_OK;
    }
    sv_state::Pending pr{};
    pr.rec.kind = SV_SWEEP_PASS;
    pr.rec.k = __builtin_popcountll(w.qmask);
    pr.rec.c = 0;
    pr.rec.lowest_target = lo;
    pr.rec.highest_target = hi;
    pr.rec.num_gates = w.ngates;
    pr.rec.bytes = 2.0 * double(h->bytes);
    // every block a dense 16 x 16 complex matrix: 8 * 16 - 2 flops per
    // amplitude; on the matrix cores three real products of 2 * 16 flops
    // per amplitude each (FP32 / FP64), or with split BF16 operands two
    // real output rows x 32 terms x six part products x 2 flops (BF16)
    pr.rec.flops = double(nsub) * (8.0 * 16.0 - 2.0) * std::ldexp(1.0, h->n);
    pr.rec.mfma_flops = double(nsub) * (w.split ? 768.0 : 96.0) * std::ldexp(1.0, h->n);
    pr.rec.precision = w.split ? SV_PREC_BF16X6 : SV_PREC_NATIVE;
    pr.rec.blocks = int(nsub);
    for (size_t i = 0; i < nsub; ++i) {
        pr.rec.term_blocks += (!w.front[i].empty() || !w.back[i].empty()) ? 1 : 0;
        pr.rec.variant_blocks += w.vq[i] != 0 ? 1 : 0;
    }
    pr.rec.tile_log = T;
    for (int b = 0; b < T; ++b)
        pr.rec.tile_mask |= uint64_t(1) << tb[b];
    int rc = prof_begin(h, pr);
    if (rc != SV_OK)
        return rc;
    const char *base = static_cast<const char *>(h->d_arena);
    bool phases = false;
    for (size_t i = 0; i < nsub; ++i)
        phases = phases || !w.front[i].empty() || !w.back[i].empty();
    hipError_t e =
        launch_pass(h->d_state, h->n, h->dtype, T, tb, base + w.off, int(nsub), base, phases, w.split, h->stream);
    if (e != hipSuccess) {
        set_error("pass %zu launch failed: %s", index, hipGetErrorString(e));
        return SV_EDEVICE;
    }
    rc = prof_end(h, pr);
    if (rc != SV_OK)
        return rc;
    acc.sweeps += 1;
    if (w.ngates > 1)
        acc.fused_blocks += 1;
    acc.algorithmic_bytes += pr.rec.bytes;
    acc.flops += pr.rec.flops;
    return SV_OK;
}

// Run a circuit as LDS passes (SV_PLAN_PASSES), fused, uploaded and launched
// in chunks of 1, 2, 4, ... passes as in run_groups.
// Run a pass plan (plan_passes or the learned planner) on the gate list it
// was made for (the circuit with diagonal pairs pre-fused).
int run_pass_plan(sv_state *h, const std::vector<Block> &gates, const std::vector<PassGroup> &pg, int precision,
                  int ngates, sv_run_stats *st)
{
    const uint64_t S = amp_bytes(h->dtype);
    const uint64_t mat16 = (256 * S + 255) & ~uint64_t(255);
    std::vector<PassWork> work(pg.size());
    uint64_t total = 0;
    for (size_t i = 0; i < pg.size(); ++i) {
        PassWork &w = work[i];
        static_cast<PassGroup &>(w) = pg[i];
        w.split = precision == SV_PREC_BF16X6 && h->dtype == SV_C64;
        w.off = total;
        if (w.kernel) {
            uint64_t nmat = 0;
            for (size_t j = 0; j < w.subs.size(); ++j) {
                w.nterm_max += uint64_t(1 << kMaxPhaseQubits) * (w.front[j].size() + w.back[j].size());
                nmat += uint64_t(1) << __builtin_popcountll(w.vq[j]);
            }
            // the launch runs the phase-free kernel exactly when no block has
            // phase gates (stage_launch_pass)
            w.presplit = w.split && w.nterm_max == 0;
            w.bytes = ((w.subs.size() * sizeof(PassSub) + 255) & ~uint64_t(255)) +
                      ((w.nterm_max * sizeof(PassTerm) + 255) & ~uint64_t(255)) +
                      nmat * (w.presplit ? kPresplitBytes : mat16);
        } else {
            for (const Group &g : w.subs) {
                const Block &first = gates[size_t(g.members[0])];
                const int k = g.members.size() == 1 ? first.k : __builtin_popcountll(g.qmask);
                const int c = g.members.size() == 1 ? first.c : 0;
                w.bytes += matrix_bytes(h, (k == 3 && pads_to_four(h->n, h->dtype, c, precision)) ? 4 : k);
            }
        }
        total += w.bytes;
    }
    int rc = ensure_arena(h, total);
    if (rc != SV_OK)
        return rc;
    sv_run_stats acc{};
    acc.gates = ngates;
    std::vector<const Block *> mp;
    std::vector<Block> sweeps;
    std::vector<std::vector<Block>> chunk_sweeps;
    for (size_t next = 0, size = 1; next < work.size() && rc == SV_OK; next += size, size *= 2) {
        const size_t end = std::min(work.size(), next + size);
        chunk_sweeps.assign(end - next, std::vector<Block>());
        for (size_t i = next; i < end && rc == SV_OK; ++i) {
            const PassWork &w = work[i];
            if (w.kernel) {
                rc = stage_launch_pass(h, gates, w, false, i, acc);
                continue;
            }
            uint64_t off = w.off;
            for (const Group &g : w.subs) {
                mp.clear();
                for (int m : g.members)
                    mp.push_back(&gates[size_t(m)]);
                Block b = fuse(mp, g.qmask);
                if (padded_exec(h, b, precision))
                    b = pad_to_four(h, b);
                if (b.k >= 2)
                    stage_matrix(h, b, off);
                off += matrix_bytes(h, b.k);
                chunk_sweeps[i - next].push_back(std::move(b));
            }
        }
        if (rc != SV_OK)
            break;
        rc = upload_range(h, work[next].off, end < work.size() ? work[end].off : total);
        for (size_t i = next; i < end && rc == SV_OK; ++i) {
            const PassWork &w = work[i];
            if (w.kernel) {
                rc = stage_launch_pass(h, gates, w, true, i, acc);
                continue;
            }
            uint64_t off = w.off;
            for (const Block &b : chunk_sweeps[i - next]) {
                if (rc != SV_OK)
                    break;
                rc = launch_block(h, b, static_cast<const char *>(h->d_arena) + off, precision, i, acc);
                off += matrix_bytes(h, b.k);
            }
        }
    }
    if (total > 0) {
        HIP_TRY(hipEventRecord(h->arena_done, h->stream));
        h->arena_pending = true;
    }
    if (rc == SV_OK && st)
        *st = acc;
    return rc;
}

int parse_pauli(const sv_state *h, const char *term, uint64_t &x, uint64_t &yz, int &ny)
{
    if (term == nullptr) {
        set_error("NULL Pauli term");
        return SV_EINVAL;
    }
    const size_t len = strlen(term);
    if (len != size_t(h->n)) {
        set_error("Pauli term of length %zu on a %d-qubit state", len, h->n);
        return SV_EINVAL;
    }
    x = yz = 0;
    ny = 0;
    for (int q = 0; q < h->n; ++q) {
        const uint64_t bit = uint64_t(1) << h->qmap[q];
        switch (term[q]) {
        case 'I': case 'i': break;
        case 'X': case 'x': x |= bit; break;
        case 'Y': case 'y': x |= bit; yz |= bit; ++ny; break;
        case 'Z': case 'z': yz |= bit; break;
        default:
            set_error("bad Pauli character '%c'", term[q]);
            return SV_EINVAL;
        }
    }
    return SV_OK;
}

int max_device_bytes_env(uint64_t &limit)
{
    const char *e = getenv("SV_MAX_DEVICE_BYTES");
    if (!e || !*e)
        return 0;
    limit = strtoull(e, nullptr, 10);
    return 1;
}

}  // namespace

extern "C" {

const char *sv_last_error(void)
{
    return g_error.c_str();
}

int sv_state_bytes(int n, int dtype, uint64_t *bytes)
{
    if (n < 1 || n > SV_MAX_QUBITS) {
        set_error("qubit count %d outside 1..%d", n, SV_MAX_QUBITS);
        return SV_EINVAL;
    }
    if (dtype != SV_C64 && dtype != SV_C128) {
        set_error("unknown dtype %d", dtype);
        return SV_EINVAL;
    }
    if (!bytes) {
        set_error("NULL output");
        return SV_EINVAL;
    }
    *bytes = (uint64_t(1) << n) * amp_bytes(dtype);
    return SV_OK;
}

static int init_handle(sv_state *h)
{
    for (int q = 0; q < SV_MAX_QUBITS; ++q)
        h->qmap[q] = q;
    HIP_TRY(hipEventCreateWithFlags(&h->arena_done, hipEventDisableTiming));
    hipError_t e = launch_reset(h->d_state, h->n, h->dtype, h->stream);
    if (e != hipSuccess) {
        set_error("reset launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    return SV_OK;
}

int sv_create(int n, int dtype, sv_handle *out)
{
    clear_error();
    uint64_t bytes = 0;
    int rc = sv_state_bytes(n, dtype, &bytes);
    if (rc != SV_OK)
        return rc;
    if (!out) {
        set_error("NULL output handle");
        return SV_EINVAL;
    }
    uint64_t limit = 0;
    if (max_device_bytes_env(limit) && bytes > limit) {
        set_error("state of %llu bytes exceeds SV_MAX_DEVICE_BYTES=%llu", (unsigned long long)bytes,
                  (unsigned long long)limit);
        return SV_ENOMEM;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    size_t freeb = 0, totalb = 0;
    HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    if (bytes > freeb) {
        set_error("state of %llu bytes does not fit in %llu free bytes", (unsigned long long)bytes,
                  (unsigned long long)freeb);
        return SV_ENOMEM;
    }
    sv_state *h = new (std::nothrow) sv_state();
    if (!h) {
        set_error("out of host memory");
        return SV_ENOMEM;
    }
    h->n = n;
    h->dtype = dtype;
    h->bytes = bytes;
    h->device = dev;
    if (hipMalloc(&h->d_state, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        set_error("hipMalloc of %llu bytes failed", (unsigned long long)bytes);
        return SV_ENOMEM;
    }
    h->owned = true;
    rc = init_handle(h);
    if (rc != SV_OK) {
        sv_destroy(h);
        return rc;
    }
    *out = h;
    return SV_OK;
}

int sv_create_on(void *device_ptr, uint64_t bytes, int n, int dtype, void *stream, sv_handle *out)
{
    clear_error();
    uint64_t need = 0;
    int rc = sv_state_bytes(n, dtype, &need);
    if (rc != SV_OK)
        return rc;
    if (!out || !device_ptr) {
        set_error("NULL pointer argument");
        return SV_EINVAL;
    }
    if (bytes < need) {
        set_error("buffer of %llu bytes is smaller than the %llu-byte state", (unsigned long long)bytes,
                  (unsigned long long)need);
        return SV_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(device_ptr) % 16 != 0) {
        set_error("device buffer must be 16-byte aligned");
        return SV_EINVAL;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    sv_state *h = new (std::nothrow) sv_state();
    if (!h) {
        set_error("out of host memory");
        return SV_ENOMEM;
    }
    h->n = n;
    h->dtype = dtype;
    h->bytes = need;
    h->device = dev;
    h->d_state = device_ptr;
    h->owned = false;
    h->stream = static_cast<hipStream_t>(stream);
    rc = init_handle(h);
    if (rc != SV_OK) {
        sv_destroy(h);
        return rc;
    }
    *out = h;
    return SV_OK;
}

int sv_destroy(sv_handle h)
{
    if (!h)
        return SV_OK;
    DeviceGuard g(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->owned && h->d_state)
        (void)hipFree(h->d_state);
    if (h->d_scratch)
        (void)hipFree(h->d_scratch);
    if (h->d_arena)
        (void)hipFree(h->d_arena);
    if (h->h_pinned)
        (void)hipHostFree(h->h_pinned);
    if (h->h_arena)
        (void)hipHostFree(h->h_arena);
    if (h->arena_done)
        (void)hipEventDestroy(h->arena_done);
    for (hipEvent_t e : h->ev_pool)
        (void)hipEventDestroy(e);
    delete h;
    return SV_OK;
}

int sv_set_stream(sv_handle h, void *stream)
{
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    h->stream = static_cast<hipStream_t>(stream);
    return SV_OK;
}

int sv_synchronize(sv_handle h)
{
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    DeviceGuard g(h->device);
    HIP_TRY(hipStreamSynchronize(h->stream));
    return SV_OK;
}

int sv_reset(sv_handle h)
{
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    DeviceGuard g(h->device);
    for (int q = 0; q < SV_MAX_QUBITS; ++q)
        h->qmap[q] = q;
    hipError_t e = launch_reset(h->d_state, h->n, h->dtype, h->stream);
    if (e != hipSuccess) {
        set_error("reset launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    return SV_OK;
}

int sv_apply_gate(sv_handle h, const double *U, const int *targets, int k, const int *controls, int c)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (!U || !targets || (c > 0 && !controls) || k < 1 || k > SV_MAX_TARGETS || c < 0 ||
        c > SV_MAX_CONTROLS) {
        set_error("bad gate arguments (k=%d, c=%d)", k, c);
        return SV_EINVAL;
    }
    sv_gate g{};
    g.kind = SV_GATE_MATRIX;
    g.num_targets = k;
    g.num_controls = c;
    for (int j = 0; j < k; ++j)
        g.targets[j] = targets[j];
    for (int j = 0; j < c; ++j)
        g.controls[j] = controls[j];
    g.matrix = U;
    rc = validate_gate(g, h->n, 0);
    if (rc != SV_OK)
        return rc;
    std::vector<Block> blocks(1, gate_block(g));
    DeviceGuard dg(h->device);
    return run_blocks(h, blocks, SV_PREC_NATIVE, 1, nullptr);
}

// Whether opts.pass_tile names a tile the pass kernels have for this state.
static bool pass_tile_allowed(const sv_state *h, const sv_plan_opts &o)
{
    const int T0 = pass_tile_log(h->dtype);
    if (o.pass_tile == T0)
        return true;
    const bool split = h->dtype == SV_C64 && o.precision == SV_PREC_BF16X6;
    return o.pass_tile == T0 + 1 && !split && h->n >= T0 + 1;
}

static void key_gates(std::vector<uint64_t> &key, const std::vector<Block> &gates)
{
    key.push_back(gates.size());
    for (const Block &b : gates) {
        uint64_t t = 0, c = 0;
        for (int j = 0; j < b.k; ++j)
            t |= uint64_t(b.targets[j]) << (6 * j);
        for (int j = 0; j < b.c; ++j)
            c |= uint64_t(b.controls[j]) << (6 * j);
        key.push_back(uint64_t(b.k) | uint64_t(b.c) << 4 | uint64_t(b.diag) << 8 | uint64_t(is_phase_gate(b)) << 9 |
                      uint64_t(uint32_t(b.ngates)) << 16);
        key.push_back(t);
        key.push_back(c);
    }
}

// Everything a plan for this circuit on this handle depends on.
static std::vector<uint64_t> plan_key(const sv_state *h, const sv_plan_opts &o, const std::vector<Block> &gates,
                                      const std::vector<Block> &pre)
{
    std::vector<uint64_t> key;
    key.reserve(8 + h->n + 3 * (gates.size() + pre.size()));
    key.push_back(uint64_t(uint32_t(o.mode)));
    key.push_back(uint64_t(uint32_t(o.max_fused)) | uint64_t(uint32_t(o.precision)) << 8 |
                  uint64_t(uint32_t(o.pass_qubits)) << 16 | uint64_t(uint32_t(o.pass_orders)) << 24 |
                  uint64_t(uint32_t(o.pass_tile)) << 40);
    key.push_back(uint64_t(h->n) | uint64_t(h->dtype) << 8);
    if (o.mode == SV_PLAN_LEARNED) {
        key.push_back(uint64_t(reinterpret_cast<uintptr_t>(h->model)));
        key.push_back(costmodel_version(h->model));
    }
    for (int q = 0; q < h->n; ++q)
        key.push_back(uint64_t(h->qmap[q]));
    if (o.mode == SV_PLAN_LEARNED)
        key_gates(key, gates);
    key_gates(key, pre);
    return key;
}

static PlanCacheEntry *find_plan(sv_state *h, const std::vector<uint64_t> &key)
{
    for (size_t i = 0; i < h->plan_cache.size(); ++i)
        if (h->plan_cache[i].key == key) {
            if (i > 0)
                std::rotate(h->plan_cache.begin(), h->plan_cache.begin() + long(i), h->plan_cache.begin() + long(i) + 1);
            return &h->plan_cache.front();
        }
    return nullptr;
}

static PlanCacheEntry *keep_plan(sv_state *h, PlanCacheEntry &&e)
{
    constexpr size_t kPlansKept = 4;
    h->plan_cache.insert(h->plan_cache.begin(), std::move(e));
    if (h->plan_cache.size() > kPlansKept)
        h->plan_cache.pop_back();
    return &h->plan_cache.front();
}

int sv_apply_circuit(sv_handle h, const sv_gate *gates, int ngates, const sv_plan_opts *opts, sv_run_stats *stats)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    sv_plan_opts o{};
    if (opts)
        o = *opts;
    // gates as one-gate blocks (validated), then grouped by the plan mode
    sv_plan_opts plain = o;
    plain.mode = SV_PLAN_PLAIN;
    plain.pass_qubits = 0;
    plain.pass_orders = 0;
    plain.pass_tile = 0;
    std::vector<Block> gates_b;
    rc = plan_circuit(h->n, h->dtype, gates, ngates, plain, gates_b);
    if (rc != SV_OK)
        return rc;
    if (o.mode < SV_PLAN_PLAIN || o.mode > SV_PLAN_PASSES) {
        set_error("unknown plan mode %d", o.mode);
        return SV_EINVAL;
    }
    if (o.mode != SV_PLAN_PLAIN && (o.max_fused < 1 || o.max_fused > SV_MAX_TARGETS)) {
        set_error("max_fused %d outside 1..%d", o.max_fused, SV_MAX_TARGETS);
        return SV_EINVAL;
    }
    if (o.mode == SV_PLAN_PASSES ? (o.pass_qubits != 0 && (o.pass_qubits < 4 || o.pass_qubits > kMaxPassQubits))
                                 : o.pass_qubits != 0) {
        set_error("pass_qubits %d: 4..%d (0 for %d) with SV_PLAN_PASSES, else 0", o.pass_qubits, kMaxPassQubits,
                  kMaxPassQubits);
        return SV_EINVAL;
    }
    if (o.mode == SV_PLAN_PASSES ? (o.pass_orders < -1 || o.pass_orders > kMaxPassOrders) : o.pass_orders != 0) {
        set_error("pass_orders %d: -1..%d with SV_PLAN_PASSES, else 0", o.pass_orders, kMaxPassOrders);
        return SV_EINVAL;
    }
    if (o.pass_tile != 0 && (o.mode != SV_PLAN_PASSES || !pass_tile_allowed(h, o))) {
        set_error("pass_tile %d: 0, or with SV_PLAN_PASSES the smallest pass tile or (except complex64 split-BF16 "
                  "blocks) twice it", o.pass_tile);
        return SV_EINVAL;
    }
    DeviceGuard dg(h->device);
    if (o.mode == SV_PLAN_PASSES || (o.mode == SV_PLAN_LEARNED && h->model)) {
        const std::vector<Block> pre = prefuse_diagonal_pairs(gates_b);
        const std::vector<uint64_t> key = plan_key(h, o, gates_b, pre);
        PlanCacheEntry *e = find_plan(h, key);
        if (e == nullptr) {
            PlanCacheEntry ne;
            ne.key = key;
            if (o.mode == SV_PLAN_PASSES) {
                ne.plan = plan_passes(pre, o.pass_qubits ? o.pass_qubits : kMaxPassQubits, o.max_fused, h->n,
                                      pass_tile_log(h->dtype), h->qmap, o.pass_orders);
                for (PassGroup &w : ne.plan)
                    if (w.kernel)
                        w.tile_log = o.pass_tile;
            } else {
                rc = rank_plans(h->model, h->n, h->dtype, gates_b, o.max_fused, o.precision, ne.width, nullptr,
                                h->qmap, &ne.plan);
                if (rc != SV_OK)
                    return rc;
            }
            e = keep_plan(h, std::move(ne));
        }
        if (o.mode == SV_PLAN_PASSES || e->width == 0)
            return run_pass_plan(h, pre, e->plan, o.precision, ngates, stats);
        return run_groups(h, gates_b, group_greedy(gates_b, e->width), o.precision, ngates, stats);
    }
    std::vector<Group> groups;
    if (o.mode == SV_PLAN_PLAIN) {
        groups.reserve(gates_b.size());
        for (size_t i = 0; i < gates_b.size(); ++i)
            groups.push_back(Group{std::vector<int>(1, int(i)), qubit_mask(gates_b[i])});
    } else {
        groups = group_greedy(gates_b, o.max_fused);
    }
    return run_groups(h, gates_b, groups, o.precision, ngates, stats);
}

int sv_set_costmodel(sv_handle h, sv_costmodel_handle m)
{
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    h->model = m;
    return SV_OK;
}

int sv_swap_bits(sv_handle h, int lo, int hi, int width)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (width < 1 || width > 6 || lo < 0 || lo + width > hi || hi + width > h->n) {
        set_error("bad bit fields lo=%d hi=%d width=%d for n=%d", lo, hi, width, h->n);
        return SV_EINVAL;
    }
    DeviceGuard dg(h->device);
    sv_state::Pending pr{};
    pr.rec.kind = SV_SWEEP_BITSWAP;
    pr.rec.k = width;
    pr.rec.lowest_target = lo;
    pr.rec.highest_target = hi;
    pr.rec.bytes = 2.0 * double(h->bytes) * (1.0 - std::ldexp(1.0, -width));
    rc = prof_begin(h, pr);
    if (rc != SV_OK)
        return rc;
    hipError_t e = launch_bitswap(h->d_state, h->n, h->dtype, lo, hi, width, h->stream);
    if (e != hipSuccess) {
        set_error("bit swap launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    rc = prof_end(h, pr);
    if (rc != SV_OK)
        return rc;
    for (int q = 0; q < h->n; ++q) {
        const int p = h->qmap[q];
        if (p >= lo && p < lo + width)
            h->qmap[q] = p - lo + hi;
        else if (p >= hi && p < hi + width)
            h->qmap[q] = p - hi + lo;
    }
    return SV_OK;
}

int sv_qubit_map(sv_handle h, int *map)
{
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (!map) {
        set_error("NULL map");
        return SV_EINVAL;
    }
    for (int q = 0; q < h->n; ++q)
        map[q] = h->qmap[q];
    return SV_OK;
}

int sv_probabilities(sv_handle h, const int *qubits, int m, double *out)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (m < 0 || m > h->n || m > 30 || !out || (m > 0 && !qubits)) {
        set_error("bad marginal request (m=%d, n=%d)", m, h->n);
        return SV_EINVAL;
    }
    int phys[30];
    uint64_t used = 0;
    for (int b = 0; b < m; ++b) {
        if (qubits[b] < 0 || qubits[b] >= h->n || ((used >> qubits[b]) & 1)) {
            set_error("bad or repeated qubit %d", qubits[b]);
            return SV_EINVAL;
        }
        used |= uint64_t(1) << qubits[b];
        phys[b] = h->qmap[qubits[b]];
    }
    DeviceGuard dg(h->device);
    const uint64_t nbins = uint64_t(1) << m;
    const uint64_t part = marginal_scratch_doubles(h->n, m, phys);
    rc = ensure_scratch(h, (part + nbins) * sizeof(double));
    if (rc != SV_OK)
        return rc;
    rc = ensure_pinned(h, nbins * sizeof(double));
    if (rc != SV_OK)
        return rc;
    double *d_out = h->d_scratch + part;
    hipError_t e = launch_marginal(h->d_state, h->n, h->dtype, phys, m, h->d_scratch, d_out, h->stream);
    if (e != hipSuccess) {
        set_error("marginal launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    HIP_TRY(hipMemcpyAsync(h->h_pinned, d_out, nbins * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    memcpy(out, h->h_pinned, nbins * sizeof(double));
    return SV_OK;
}

// Expectation values of parsed Pauli strings (x mask, y|z mask, number of
// Y) on the handle's stream: d_part holds the launches' partial sums
// (expect_scratch_doubles), d_res 2 * nterms result doubles, h_res as many
// host doubles (pinned or not), order[nterms] an index buffer.  Device
// results: the Z-only strings first (one double each, in order of
// appearance), then (Re, Im) of each general string.  Every launch is
// queued, then one copy and one wait.
static int expect_core(sv_state *h, int nterms, const uint64_t *xs, const uint64_t *yzs, const int *nys,
                       double *d_part, double *d_res, double *h_res, int *order, double *out)
{
    int nz = 0;
    for (int t = 0; t < nterms; ++t)
        if (xs[t] == 0)
            order[nz++] = t;
    int nxy = 0;
    for (int t = 0; t < nterms; ++t)
        if (xs[t] != 0)
            order[nz + nxy++] = t;
    constexpr int kZ = 64;
    const int zb = std::min(expect_z_batch(), kZ);
    for (int s = 0; s < nz; s += zb) {
        const int nb = std::min(zb, nz - s);
        uint64_t z[kZ];
        for (int j = 0; j < nb; ++j)
            z[j] = yzs[order[s + j]];
        hipError_t e = launch_expect_z(h->d_state, h->n, h->dtype, z, nb, d_part, d_res + s, h->stream);
        if (e != hipSuccess) {
            set_error("Z expectation launch failed: %s", hipGetErrorString(e));
            return SV_EDEVICE;
        }
    }
    for (int q = 0; q < nxy; ++q) {
        const int t = order[nz + q];
        hipError_t e = launch_expect_xy(h->d_state, h->n, h->dtype, xs[t], yzs[t], d_part, d_res + nz + 2 * q,
                                        h->stream);
        if (e != hipSuccess) {
            set_error("Pauli expectation launch failed: %s", hipGetErrorString(e));
            return SV_EDEVICE;
        }
    }
    const size_t nres = size_t(nz) + 2 * size_t(nxy);
    HIP_TRY(hipMemcpyAsync(h_res, d_res, nres * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int j = 0; j < nz; ++j)
        out[order[j]] = h_res[j];
    static const cd ipow[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    for (int q = 0; q < nxy; ++q) {
        const int t = order[nz + q];
        const cd S(h_res[nz + 2 * q], h_res[nz + 2 * q + 1]);
        // multiply by i^(number of Y)
        out[t] = (ipow[nys[t] & 3] * S).real();
    }
    return SV_OK;
}

int sv_expect_pauli(sv_handle h, const char *const *terms, int nterms, double *out)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (nterms < 0 || (nterms > 0 && (!terms || !out))) {
        set_error("bad term list");
        return SV_EINVAL;
    }
    std::vector<uint64_t> xs(nterms), yzs(nterms);
    std::vector<int> nys(nterms), order(nterms);
    for (int t = 0; t < nterms; ++t) {
        rc = parse_pauli(h, terms[t], xs[t], yzs[t], nys[t]);
        if (rc != SV_OK)
            return rc;
    }
    if (nterms == 0)
        return SV_OK;
    DeviceGuard dg(h->device);
    const uint64_t part = expect_scratch_doubles(h->n);
    // result slots: 2 doubles per term
    rc = ensure_scratch(h, (part + 2 * uint64_t(nterms)) * sizeof(double));
    if (rc != SV_OK)
        return rc;
    rc = ensure_pinned(h, 2 * uint64_t(nterms) * sizeof(double));
    if (rc != SV_OK)
        return rc;
    return expect_core(h, nterms, xs.data(), yzs.data(), nys.data(), h->d_scratch, h->d_scratch + part,
                       static_cast<double *>(h->h_pinned), order.data(), out);
}

int sv_expect_pauli_noalloc(sv_handle h, const char *const *terms, int nterms, double *out)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (nterms < 0 || nterms > SV_NOALLOC_MAX_TERMS || (nterms > 0 && (!terms || !out))) {
        set_error("bad term list (nterms %d, at most %d without allocation)", nterms, SV_NOALLOC_MAX_TERMS);
        return SV_EINVAL;
    }
    // fixed-size host workspace: nothing is allocated on the success path
    uint64_t xs[SV_NOALLOC_MAX_TERMS], yzs[SV_NOALLOC_MAX_TERMS];
    int nys[SV_NOALLOC_MAX_TERMS], order[SV_NOALLOC_MAX_TERMS];
    double h_res[2 * SV_NOALLOC_MAX_TERMS];
    for (int t = 0; t < nterms; ++t) {
        rc = parse_pauli(h, terms[t], xs[t], yzs[t], nys[t]);
        if (rc != SV_OK)
            return rc;
    }
    if (nterms == 0)
        return SV_OK;
    DeviceGuard dg(h->device);
    double *d_scr = nullptr;
    uint64_t have = 0;
    rc = noalloc_scratch(h->device, &d_scr, &have);
    if (rc != SV_OK)
        return rc;
    const uint64_t part = expect_scratch_doubles(h->n);
    if (part + 2 * uint64_t(nterms) > have) {
        set_error("fixed scratch of %llu doubles is too small", (unsigned long long)have);
        return SV_EUNSUPPORTED;
    }
    return expect_core(h, nterms, xs, yzs, nys, d_scr, d_scr + part, h_res, order, out);
}

// Check a shot request: shots >= 0, uniforms in [0, 1).
static int check_shots(const double *uniforms, int shots, const int64_t *out)
{
    if (shots < 0 || (shots > 0 && (!uniforms || !out))) {
        set_error("bad sampling arguments");
        return SV_EINVAL;
    }
    for (int s = 0; s < shots; ++s)
        if (!(uniforms[s] >= 0.0 && uniforms[s] < 1.0)) {
            set_error("uniform %d = %g outside [0, 1)", s, uniforms[s]);
            return SV_EINVAL;
        }
    return SV_OK;
}

// Shot work area in device scratch: blocks (int64) | targets | outputs
// (int64) | uniforms, shots entries each.
constexpr uint64_t kShotWork = 4;

// Queue the shots from the totals d_bs[0..nb) of consecutive 2^lbs-amplitude
// blocks, all on the device: the uniforms go up through the pinned staging
// (its first shots * 8 bytes, so no copy into it may be pending), each shot's
// block and residual target are chosen from the totals, then the in-block
// search writes physical indices to the outputs.  Returns the outputs.
static int queue_samples(sv_state *h, const double *d_bs, uint64_t nb, int lbs, const double *uniforms, int shots,
                         double *d_work, int64_t **d_out)
{
    int64_t *d_blk = reinterpret_cast<int64_t *>(d_work);
    double *d_tgt = d_work + shots;
    *d_out = reinterpret_cast<int64_t *>(d_work + 2 * uint64_t(shots));
    double *d_uni = d_work + 3 * uint64_t(shots);
    memcpy(h->h_pinned, uniforms, uint64_t(shots) * 8);
    HIP_TRY(hipMemcpyAsync(d_uni, h->h_pinned, uint64_t(shots) * 8, hipMemcpyHostToDevice, h->stream));
    hipError_t e = launch_sample_prep(d_bs, nb, d_uni, shots, d_blk, d_tgt, h->stream);
    if (e == hipSuccess)
        e = launch_sample_search(h->d_state, h->n, h->dtype, d_blk, d_tgt, shots, *d_out, lbs, h->stream);
    if (e != hipSuccess) {
        set_error("sampling launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    return SV_OK;
}

// Physical sample indices (copied back) to logical ones.
static void map_samples(const sv_state *h, const int64_t *phys, int shots, int64_t *out)
{
    const bool ident = identity_map(h);
    for (int s = 0; s < shots; ++s) {
        if (ident) {
            out[s] = phys[s];
        } else {
            int64_t l = 0;
            for (int q = 0; q < h->n; ++q)
                l |= ((phys[s] >> h->qmap[q]) & 1) << q;
            out[s] = l;
        }
    }
}

int sv_sample(sv_handle h, const double *uniforms, int shots, int64_t *out)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    rc = check_shots(uniforms, shots, out);
    if (rc != SV_OK || shots == 0)
        return rc;
    DeviceGuard dg(h->device);
    const int lbs = sample_log_block(h->n);
    const uint64_t nb = uint64_t(1) << (h->n - lbs);
    // scratch: block sums | shot work; pinned: the uniforms, then the outputs
    rc = ensure_scratch(h, (nb + kShotWork * uint64_t(shots)) * 8);
    if (rc != SV_OK)
        return rc;
    rc = ensure_pinned(h, uint64_t(shots) * 8);
    if (rc != SV_OK)
        return rc;
    double *d_bs = h->d_scratch;
    hipError_t e = launch_block_sums(h->d_state, h->n, h->dtype, d_bs, h->stream);
    if (e != hipSuccess) {
        set_error("block-sum launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    int64_t *d_out = nullptr;
    rc = queue_samples(h, d_bs, nb, lbs, uniforms, shots, h->d_scratch + nb, &d_out);
    if (rc != SV_OK)
        return rc;
    HIP_TRY(hipMemcpyAsync(h->h_pinned, d_out, uint64_t(shots) * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    map_samples(h, static_cast<const int64_t *>(h->h_pinned), shots, out);
    return SV_OK;
}

int sv_readout(sv_handle h, const int *qubits, int m, double *probs, const char *const *terms, int nterms,
               double *expect, const double *uniforms, int shots, int64_t *samples)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (m < 0 || m > h->n || m > 30 || (probs && m > 0 && !qubits) || (!probs && m != 0)) {
        set_error("bad marginal request (m=%d, n=%d)", m, h->n);
        return SV_EINVAL;
    }
    int phys[30];
    uint64_t used = 0;
    for (int b = 0; b < m; ++b) {
        if (qubits[b] < 0 || qubits[b] >= h->n || ((used >> qubits[b]) & 1)) {
            set_error("bad or repeated qubit %d", qubits[b]);
            return SV_EINVAL;
        }
        used |= uint64_t(1) << qubits[b];
        phys[b] = h->qmap[qubits[b]];
    }
    if (nterms < 0 || (nterms > 0 && (!terms || !expect))) {
        set_error("bad term list");
        return SV_EINVAL;
    }
    std::vector<uint64_t> xs(nterms), zs(nterms);
    bool z_only = nterms <= kReadoutMaxZ;
    for (int t = 0; t < nterms; ++t) {
        int ny = 0;
        rc = parse_pauli(h, terms[t], xs[t], zs[t], ny);
        if (rc != SV_OK)
            return rc;
        z_only = z_only && xs[t] == 0;
    }
    rc = check_shots(uniforms, shots, samples);
    if (rc != SV_OK)
        return rc;
    const bool want_p = probs != nullptr;
    if (!want_p && nterms == 0 && shots == 0)
        return SV_OK;
    // one read of the state where the marginal's fold route allows it and
    // every string is a Z string; else the three read-outs one after another
    if (!z_only || !readout_fusable(h->n, want_p ? m : 0, phys, h->dtype) || (want_p && m == 0)) {
        if (want_p && (rc = sv_probabilities(h, qubits, m, probs)) != SV_OK)
            return rc;
        if (nterms > 0 && (rc = sv_expect_pauli(h, terms, nterms, expect)) != SV_OK)
            return rc;
        if (shots > 0 && (rc = sv_sample(h, uniforms, shots, samples)) != SV_OK)
            return rc;
        return SV_OK;
    }
    DeviceGuard dg(h->device);
    const int mm = want_p ? m : 0;
    const int lbs = readout_log_block(h->n, mm, phys, h->dtype);
    const uint64_t nb = uint64_t(1) << (h->n - lbs);
    const uint64_t nbins = want_p ? uint64_t(1) << m : 0;
    const uint64_t red = readout_scratch_doubles(h->n, mm, phys, h->dtype);
    // scratch: fold and Z partials | block totals | marginal | Z values | shot work
    const uint64_t need = red + nb + nbins + uint64_t(nterms) + kShotWork * uint64_t(shots);
    rc = ensure_scratch(h, need * 8);
    if (rc != SV_OK)
        return rc;
    // pinned: the uniforms going up; then marginal | Z values | shots coming back
    const uint64_t nres = nbins + uint64_t(nterms);
    rc = ensure_pinned(h, (nres + uint64_t(shots)) * 8);
    if (rc != SV_OK)
        return rc;
    double *d_tot = h->d_scratch + red;
    double *d_marg = d_tot + nb;
    double *d_z = d_marg + nbins;
    double *d_work = d_z + nterms;
    hipError_t e = launch_readout(h->d_state, h->n, h->dtype, phys, mm, zs.data(), nterms, h->d_scratch,
                                  want_p ? d_marg : nullptr, d_z, d_tot, h->stream);
    if (e != hipSuccess) {
        set_error("read-out launch failed: %s", hipGetErrorString(e));
        return SV_EDEVICE;
    }
    int64_t *d_out = nullptr;
    if (shots > 0 && (rc = queue_samples(h, d_tot, nb, lbs, uniforms, shots, d_work, &d_out)) != SV_OK)
        return rc;
    // one copy back and one wait for all three results
    char *hp = static_cast<char *>(h->h_pinned);
    if (nres > 0)
        HIP_TRY(hipMemcpyAsync(hp, d_marg, nres * 8, hipMemcpyDeviceToHost, h->stream));
    if (shots > 0)
        HIP_TRY(hipMemcpyAsync(hp + nres * 8, d_out, uint64_t(shots) * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (want_p)
        memcpy(probs, hp, nbins * 8);
    if (nterms > 0)
        memcpy(expect, hp + nbins * 8, uint64_t(nterms) * 8);
    if (shots > 0)
        map_samples(h, reinterpret_cast<const int64_t *>(hp + nres * 8), shots, samples);
    return SV_OK;
}

// Uniform s of the shot stream of `seed`: the s-th output of SplitMix64
// (Steele, Lea, Flood, OOPSLA 2014) started from state `seed`, i.e. the mix
// function applied to seed + (s + 1) * 0x9E3779B97F4A7C15, whose top 53 bits
// scaled by 2^-53 give a double in [0, 1).  A pure function of (seed, s), so
// any range of the stream can be produced on its own.
static double shot_uniform(uint64_t seed, uint64_t s)
{
    uint64_t z = seed + (s + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return double(z >> 11) * (1.0 / 9007199254740992.0);
}

int sv_uniforms(uint64_t seed, uint64_t first, int count, double *out)
{
    clear_error();
    if (count < 0 || (count > 0 && !out)) {
        set_error("bad uniform-stream arguments");
        return SV_EINVAL;
    }
    for (int s = 0; s < count; ++s)
        out[s] = shot_uniform(seed, first + uint64_t(s));
    return SV_OK;
}

int sv_sample_seeded(sv_handle h, int shots, uint64_t seed, int64_t *out)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (shots < 0 || (shots > 0 && !out)) {
        set_error("bad sampling arguments");
        return SV_EINVAL;
    }
    std::vector<double> u(size_t(shots) + 1);
    for (int s = 0; s < shots; ++s)
        u[s] = shot_uniform(seed, uint64_t(s));
    return sv_sample(h, u.data(), shots, out);
}

int sv_copy_to_host(sv_handle h, void *dst, uint64_t first, uint64_t count)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    const uint64_t N = uint64_t(1) << h->n;
    if (!dst || first > N || count > N - first) {
        set_error("bad copy range [%llu, +%llu) of %llu", (unsigned long long)first, (unsigned long long)count,
                  (unsigned long long)N);
        return SV_EINVAL;
    }
    if (count == 0)
        return SV_OK;
    DeviceGuard dg(h->device);
    const uint64_t S = amp_bytes(h->dtype);
    if (identity_map(h)) {
        HIP_TRY(hipMemcpyAsync(dst, static_cast<const char *>(h->d_state) + first * S, count * S,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        return SV_OK;
    }
    const uint64_t chunk = uint64_t(1) << 22;
    rc = ensure_scratch(h, std::min(count, chunk) * S);
    if (rc != SV_OK)
        return rc;
    for (uint64_t done = 0; done < count; done += chunk) {
        const uint64_t c = std::min(chunk, count - done);
        hipError_t e = launch_gather_logical(h->d_state, h->d_scratch, h->n, h->dtype, h->qmap, first + done, c,
                                             h->stream);
        if (e != hipSuccess) {
            set_error("gather launch failed: %s", hipGetErrorString(e));
            return SV_EDEVICE;
        }
        HIP_TRY(hipMemcpyAsync(static_cast<char *>(dst) + done * S, h->d_scratch, c * S, hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return SV_OK;
}

int sv_copy_from_host(sv_handle h, const void *src, uint64_t first, uint64_t count)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    const uint64_t N = uint64_t(1) << h->n;
    if (!src || first > N || count > N - first) {
        set_error("bad copy range");
        return SV_EINVAL;
    }
    const bool whole = first == 0 && count == N;
    if (!identity_map(h) && !whole) {
        set_error("partial copy into a relaid-out state (qubit map not identity)");
        return SV_EINVAL;
    }
    if (count == 0)
        return SV_OK;
    DeviceGuard dg(h->device);
    const uint64_t S = amp_bytes(h->dtype);
    HIP_TRY(hipMemcpyAsync(static_cast<char *>(h->d_state) + first * S, src, count * S, hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (whole)
        for (int q = 0; q < SV_MAX_QUBITS; ++q)
            h->qmap[q] = q;
    return SV_OK;
}

int sv_profile_enable(sv_handle h, int enable)
{
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    h->profiling = enable != 0;
    return SV_OK;
}

int sv_profile_read(sv_handle h, sv_sweep_record *out, int max, int *count)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (max < 0 || (max > 0 && !out) || !count) {
        set_error("bad profile buffer");
        return SV_EINVAL;
    }
    DeviceGuard dg(h->device);
    HIP_TRY(hipStreamSynchronize(h->stream));
    int k = 0;
    for (auto &p : h->pending) {
        if (k < max) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
            out[k] = p.rec;
            out[k].ms = ms;
        }
        ++k;
    }
    *count = k;
    h->pending.clear();
    h->ev_used = 0;
    return SV_OK;
}

int sv_pass_plan_info(int n, int dtype, const sv_gate *gates, int ngates, const sv_plan_opts *opts, int64_t *out)
{
    clear_error();
    uint64_t bytes;
    int rc = sv_state_bytes(n, dtype, &bytes);
    if (rc != SV_OK)
        return rc;
    if (!out) {
        set_error("NULL output");
        return SV_EINVAL;
    }
    sv_plan_opts o{};
    o.mode = SV_PLAN_PASSES;
    o.max_fused = 5;
    if (opts)
        o = *opts;
    if (o.mode != SV_PLAN_PASSES) {
        set_error("sv_pass_plan_info describes SV_PLAN_PASSES plans");
        return SV_EINVAL;
    }
    if (o.max_fused < 1 || o.max_fused > SV_MAX_TARGETS) {
        set_error("max_fused %d outside 1..%d", o.max_fused, SV_MAX_TARGETS);
        return SV_EINVAL;
    }
    if (o.pass_qubits != 0 && (o.pass_qubits < 4 || o.pass_qubits > kMaxPassQubits)) {
        set_error("pass_qubits %d: 4..%d (0 for %d)", o.pass_qubits, kMaxPassQubits, kMaxPassQubits);
        return SV_EINVAL;
    }
    if (o.pass_orders < -1 || o.pass_orders > kMaxPassOrders) {
        set_error("pass_orders %d: -1..%d", o.pass_orders, kMaxPassOrders);
        return SV_EINVAL;
    }
    sv_plan_opts plain = o;
    plain.mode = SV_PLAN_PLAIN;
    plain.pass_qubits = 0;
    plain.pass_orders = 0;
    plain.pass_tile = 0;
    std::vector<Block> gates_b;
    rc = plan_circuit(n, dtype, gates, ngates, plain, gates_b);
    if (rc != SV_OK)
        return rc;
    const std::vector<Block> pg = prefuse_diagonal_pairs(gates_b);
    const std::vector<PassGroup> plan =
        plan_passes(pg, o.pass_qubits ? o.pass_qubits : kMaxPassQubits, o.max_fused, n, pass_tile_log(dtype), nullptr,
                    o.pass_orders);
    int64_t r[8] = {};
    std::vector<char> seen(pg.size(), 0);
    bool twice = false;
    auto cover = [&](int m) {
        twice = twice || seen[size_t(m)];
        seen[size_t(m)] = 1;
        r[6] += pg[size_t(m)].ngates;
    };
    for (const PassGroup &w : plan) {
        r[0] += 1;
        if (w.kernel) {
            r[1] += 1;
            r[2] += int64_t(w.subs.size());
            for (size_t i = 0; i < w.subs.size(); ++i) {
                r[3] += w.vq[i] != 0;
                r[4] += !w.front[i].empty() || !w.back[i].empty();
                for (int m : w.front[i])
                    cover(m);
                for (int m : w.back[i])
                    cover(m);
            }
        } else {
            r[5] += int64_t(w.subs.size());
        }
        for (const Group &g : w.subs)
            for (int m : g.members)
                cover(m);
    }
    if (twice)
        r[6] = -1;  // a gate placed twice: reported as an impossible count
    r[7] = int64_t(std::llround(pass_plan_cost(plan) * 1000.0));
    std::copy(r, r + 8, out);
    return SV_OK;
}

int sv_plan_create(int n, int dtype, const sv_gate *gates, int ngates, const sv_plan_opts *opts, sv_plan_handle *out)
{
    clear_error();
    uint64_t bytes;
    int rc = sv_state_bytes(n, dtype, &bytes);
    if (rc != SV_OK)
        return rc;
    if (!out) {
        set_error("NULL output");
        return SV_EINVAL;
    }
    sv_plan_opts o{};
    if (opts)
        o = *opts;
    sv_plan *p = new (std::nothrow) sv_plan();
    if (!p) {
        set_error("out of host memory");
        return SV_ENOMEM;
    }
    rc = plan_circuit(n, dtype, gates, ngates, o, p->blocks);
    if (rc != SV_OK) {
        delete p;
        return rc;
    }
    p->n = n;
    p->dtype = dtype;
    p->precision = o.precision;
    p->ngates = ngates;
    *out = p;
    return SV_OK;
}

int sv_plan_num_blocks(sv_plan_handle p, int *nblocks)
{
    if (!p || !nblocks) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    *nblocks = int(p->blocks.size());
    return SV_OK;
}

int sv_plan_block(sv_plan_handle p, int i, int *k, int *targets, int *c, int *controls, double *matrix,
                  int *num_gates)
{
    if (!p || i < 0 || i >= int(p->blocks.size())) {
        set_error("bad plan or block index");
        return SV_EINVAL;
    }
    const Block &b = p->blocks[i];
    if (k)
        *k = b.k;
    if (c)
        *c = b.c;
    if (targets)
        for (int j = 0; j < b.k; ++j)
            targets[j] = b.targets[j];
    if (controls)
        for (int j = 0; j < b.c; ++j)
            controls[j] = b.controls[j];
    if (matrix)
        for (size_t j = 0; j < b.U.size(); ++j) {
            matrix[2 * j] = b.U[j].real();
            matrix[2 * j + 1] = b.U[j].imag();
        }
    if (num_gates)
        *num_gates = b.ngates;
    return SV_OK;
}

int sv_apply_plan(sv_handle h, sv_plan_handle p, sv_run_stats *stats)
{
    clear_error();
    int rc = check_handle(h);
    if (rc != SV_OK)
        return rc;
    if (!p || p->n != h->n || p->dtype != h->dtype) {
        set_error("plan does not match the state (n or dtype)");
        return SV_EINVAL;
    }
    DeviceGuard dg(h->device);
    return run_blocks(h, p->blocks, p->precision, p->ngates, stats);
}

int sv_plan_destroy(sv_plan_handle p)
{
    delete p;
    return SV_OK;
}

}  // extern "C"
