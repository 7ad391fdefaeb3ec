// Host side of circuit batches: pass planning, task ordering, HIP-graph
// capture of one persistent launch, and the configuration autotuner.
//
// A circuit of q <= tile_bits qubits is one task: its whole state lives in
// LDS from |0...0> to the expectation values.  A wider circuit is cut into
// passes: each pass is a set of at most tile_bits qubits (always including the
// `low_bits` lowest, so global accesses stay contiguous) and the gates that act
// only on them, placed as early as their dependencies allow.  A pass runs as
// 2^(q - tile_bits) independent tiles.  Inside a pass gates are fused into
// one-qubit runs (fuse width 1) or blocks of at most two qubits (width 2),
// using the same greedy grouping as the sweep planner.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "sv_batch.h"
#include "sv_internal.h"

using namespace sv;

namespace {

constexpr uint32_t kSpinLimit = 1u << 21;

struct StepPlan {
    int inst;
    std::vector<int> members;  // gate indices within the circuit
    uint64_t qmask;
    uint32_t mat;              // complex offset in the matrix buffer
    int d;                     // matrix dimension
};

template <typename T>
int dev_upload(T *&dptr, const std::vector<T> &host, hipStream_t s)
{
    if (dptr) {
        (void)hipFree(dptr);
        dptr = nullptr;
    }
    const size_t bytes = std::max<size_t>(1, host.size()) * sizeof(T);
    if (hipMalloc((void **)&dptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("batch: cannot allocate %zu device bytes", bytes);
        return SV_ENOMEM;
    }
    if (!host.empty() && hipMemcpyAsync(dptr, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("batch: upload failed");
        return SV_EDEVICE;
    }
    return SV_OK;
}

}  // namespace

struct sv_batch {
    int dtype = 0;
    int ninst = 0;
    std::vector<int> q;
    std::vector<std::vector<sv_gate>> gates;      // structure + current parameters
    std::vector<std::vector<double>> matrices;   // copies of matrix gates' data
    std::vector<std::vector<uint64_t>> zmasks;
    int total_terms = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    sv_batch_config cfg{};
    bool built = false;
    // plan
    std::vector<StepPlan> steps;
    size_t mat_elems = 0;
    uint32_t ntasks = 0;
    uint32_t grid = 0;
    size_t lds = 0;
    // device buffers
    void *d_states = nullptr;
    BInst *d_inst = nullptr;
    BPass *d_pass = nullptr;
    BStep *d_steps = nullptr;
    BTask *d_tasks = nullptr;
    uint64_t *d_z = nullptr;
    double *d_part = nullptr;
    double *d_out = nullptr;
    uint32_t *d_ctr = nullptr;
    void *d_mats = nullptr;
    uint32_t nctr = 0;
    // pinned staging
    void *h_mats = nullptr;
    double *h_out = nullptr;
    uint32_t *h_err = nullptr;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
};

namespace {

void free_build(sv_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    void *bufs[] = {b->d_states, b->d_inst, b->d_pass, b->d_steps, b->d_tasks, b->d_z, b->d_part, b->d_out,
                    b->d_ctr, b->d_mats};
    for (void *p : bufs)
        if (p)
            (void)hipFree(p);
    b->d_states = nullptr;
    b->d_inst = nullptr;
    b->d_pass = nullptr;
    b->d_steps = nullptr;
    b->d_tasks = nullptr;
    b->d_z = nullptr;
    b->d_part = nullptr;
    b->d_out = nullptr;
    b->d_ctr = nullptr;
    b->d_mats = nullptr;
    if (b->h_mats)
        (void)hipHostFree(b->h_mats);
    if (b->h_out)
        (void)hipHostFree(b->h_out);
    if (b->h_err)
        (void)hipHostFree(b->h_err);
    b->h_mats = nullptr;
    b->h_out = nullptr;
    b->h_err = nullptr;
    b->built = false;
}

bool batch_gate_ok(const sv_gate &g)
{
    if (g.num_targets == 1 && g.num_controls <= 1)
        return true;
    return g.kind == SV_GATE_MATRIX && g.num_targets == 2 && g.num_controls == 0;
}

std::vector<Block> circuit_blocks(const sv_batch *b, int i)
{
    std::vector<Block> out;
    out.reserve(b->gates[i].size());
    for (const sv_gate &g : b->gates[i])
        out.push_back(gate_block(g));
    return out;
}

struct PassPlan {
    uint64_t bits = 0;
    std::vector<int> gates;
};

// As-soon-as-possible packing of a circuit into passes of <= L qubits.
std::vector<PassPlan> pack_passes(const std::vector<Block> &g, int q, int L, int low)
{
    std::vector<PassPlan> passes;
    std::vector<int> last(64, -1);
    const uint64_t lowmask = (uint64_t(1) << low) - 1;
    for (int i = 0; i < int(g.size()); ++i) {
        const uint64_t gm = qubit_mask(g[i]);
        int j0 = 0;
        for (int x = 0; x < q; ++x)
            if ((gm >> x) & 1)
                j0 = std::max(j0, last[x]);
        int j = -1;
        for (int p = std::max(j0, 0); p < int(passes.size()); ++p)
            if (__builtin_popcountll(passes[p].bits | gm | lowmask) <= L) {
                j = p;
                break;
            }
        if (j < 0) {
            passes.push_back(PassPlan());
            j = int(passes.size()) - 1;
            passes[j].bits = lowmask;
        }
        passes[j].bits |= gm;
        passes[j].gates.push_back(i);
        for (int x = 0; x < q; ++x)
            if ((gm >> x) & 1)
                last[x] = j;
    }
    if (passes.empty()) {
        passes.push_back(PassPlan());
        passes[0].bits = lowmask;
    }
    // pad every pass to exactly L tile bits with the lowest unused bits
    for (auto &p : passes)
        for (int x = 0; x < q && __builtin_popcountll(p.bits) < L; ++x)
            p.bits |= uint64_t(1) << x;
    return passes;
}

void fill_pass_bits(BPass &bp, uint64_t bits, int q)
{
    int lp = 0;
    for (int x = 0; x < q; ++x)
        if ((bits >> x) & 1) {
            bp.dep[lp] = uint64_t(1) << x;
            bp.ins[lp] = (uint64_t(1) << x) - 1;
            ++lp;
        }
    bp.lp = lp;
}

// Compute the current matrices of every step into the pinned buffer.
// The step matrices of every circuit into the pinned staging buffer: the
// circuits' gate matrices, then each step's fused product.  Circuits are
// independent and their steps contiguous, so host threads take whole
// circuits from a shared counter (each writes only its own steps' slots).
void fill_matrices(sv_batch *b)
{
    std::vector<size_t> first(size_t(b->ninst) + 1, b->steps.size());
    for (size_t k = b->steps.size(); k-- > 0;)
        first[size_t(b->steps[k].inst)] = k;
    for (int i = b->ninst - 1; i >= 0; --i)
        first[size_t(i)] = std::min(first[size_t(i)], first[size_t(i) + 1]);
    std::atomic<int> next{0};
    auto work = [&]() {
        for (int i; (i = next.fetch_add(1)) < b->ninst;) {
            const std::vector<Block> blocks = circuit_blocks(b, i);
            for (size_t k = first[size_t(i)]; k < first[size_t(i) + 1]; ++k) {
                const StepPlan &sp = b->steps[k];
                std::vector<const Block *> mem;
                for (int m : sp.members)
                    mem.push_back(&blocks[size_t(m)]);
                const Block f = fuse(mem, sp.qmask);
                const size_t dd = size_t(sp.d) * sp.d;
                if (b->dtype == SV_C64) {
                    float *dst = static_cast<float *>(b->h_mats) + 2 * size_t(sp.mat);
                    for (size_t e = 0; e < dd; ++e) {
                        dst[2 * e] = float(f.U[e].real());
                        dst[2 * e + 1] = float(f.U[e].imag());
                    }
                } else {
                    double *dst = static_cast<double *>(b->h_mats) + 2 * size_t(sp.mat);
                    for (size_t e = 0; e < dd; ++e) {
                        dst[2 * e] = f.U[e].real();
                        dst[2 * e + 1] = f.U[e].imag();
                    }
                }
            }
        }
    };
    const int nt = std::max(1, std::min({16, int(std::thread::hardware_concurrency()), b->ninst}));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t)
        pool.emplace_back(work);
    work();
    for (std::thread &t : pool)
        t.join();
}

int build(sv_batch *b)
{
    free_build(b);
    const int L = b->cfg.tile_bits, low = b->cfg.low_bits, fw = b->cfg.fuse_width;
    const size_t S = b->dtype == SV_C64 ? 8 : 16;
    std::vector<BInst> inst(b->ninst);
    std::vector<BPass> passes;
    std::vector<BStep> steps;
    std::vector<uint64_t> zs;
    b->steps.clear();
    uint64_t state_off = 0;
    int part_off = 0, out_off = 0, maxp = 0;
    uint32_t mat = 0;
    std::vector<std::vector<uint32_t>> ntiles_of(b->ninst);
    for (int i = 0; i < b->ninst; ++i) {
        const int q = b->q[i];
        const std::vector<Block> g = circuit_blocks(b, i);
        std::vector<PassPlan> pp;
        if (q <= L) {
            pp.resize(1);
            pp[0].bits = (q == 64) ? ~uint64_t(0) : ((uint64_t(1) << q) - 1);
            for (int k = 0; k < int(g.size()); ++k)
                pp[0].gates.push_back(k);
        } else {
            pp = pack_passes(g, q, L, low);
        }
        BInst &bi = inst[i];
        bi.q = q;
        bi.npasses = int(pp.size());
        bi.pass0 = int(passes.size());
        bi.nterms = int(b->zmasks[i].size());
        bi.term0 = int(zs.size());
        bi.out0 = out_off;
        out_off += bi.nterms;
        zs.insert(zs.end(), b->zmasks[i].begin(), b->zmasks[i].end());
        const uint32_t nt = q <= L ? 1u : (1u << (q - L));
        if (q > L) {
            bi.state_off = state_off;
            state_off += uint64_t(1) << q;
            bi.part0 = part_off;
            part_off += int(nt) * bi.nterms;
        }
        maxp = std::max(maxp, bi.npasses);
        for (int p = 0; p < int(pp.size()); ++p) {
            BPass bp{};
            fill_pass_bits(bp, pp[p].bits, q);
            bp.ntiles = nt;
            bp.need = uint32_t(p) * nt;
            bp.last = p + 1 == int(pp.size());
            bp.step0 = int(steps.size());
            // slot of each qubit inside the tile
            int slot[64];
            for (int x = 0, s = 0; x < q; ++x)
                if ((pp[p].bits >> x) & 1)
                    slot[x] = s++;
            std::vector<Block> pg;
            for (int k : pp[p].gates)
                pg.push_back(g[k]);
            for (const Group &gr : group_greedy(pg, fw)) {
                StepPlan sp;
                sp.inst = i;
                for (int m : gr.members)
                    sp.members.push_back(pp[p].gates[m]);
                sp.qmask = gr.qmask;
                std::vector<const Block *> mem;
                for (int m : gr.members)
                    mem.push_back(&pg[m]);
                const Block f = fuse(mem, gr.qmask);
                BStep st{};
                if (f.k == 1 && f.c == 0) {
                    st.type = 0;
                    st.a = uint8_t(slot[f.targets[0]]);
                } else if (f.k == 1 && f.c == 1) {
                    st.type = 1;
                    st.a = uint8_t(slot[f.targets[0]]);
                    st.b = uint8_t(slot[f.controls[0]]);
                } else if (f.k == 2 && f.c == 0) {
                    st.type = 2;
                    st.a = uint8_t(slot[f.targets[0]]);
                    st.b = uint8_t(slot[f.targets[1]]);
                } else {
                    set_error("batch: fused step of unsupported shape (k=%d, c=%d)", f.k, f.c);
                    return SV_EUNSUPPORTED;
                }
                sp.d = 1 << f.k;
                sp.mat = mat;
                st.mat = mat;
                mat += uint32_t(sp.d * sp.d);
                steps.push_back(st);
                b->steps.push_back(sp);
            }
            bp.nsteps = int(steps.size()) - bp.step0;
            bp.mat0 = bp.nsteps > 0 ? steps[size_t(bp.step0)].mat : mat;
            bp.nmat = mat - bp.mat0;
            passes.push_back(bp);
        }
        ntiles_of[i].assign(pp.size(), nt);
    }
    b->mat_elems = mat;
    b->total_terms = out_off;
    // tasks: level-major (pass p of every circuit before pass p+1), widest first
    std::vector<int> order(b->ninst);
    for (int i = 0; i < b->ninst; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->q[x] > b->q[y]; });
    std::vector<BTask> tasks;
    for (int p = 0; p < maxp; ++p)
        for (int i : order)
            if (p < inst[i].npasses)
                for (uint32_t t = 0; t < ntiles_of[i][p]; ++t)
                    tasks.push_back(BTask{uint32_t(i), uint32_t(p), t, 0});
    b->ntasks = uint32_t(tasks.size());

    hipStream_t s = b->stream;
    int rc;
    if (state_off > 0 && hipMalloc(&b->d_states, state_off * S) != hipSuccess) {
        (void)hipGetLastError();
        set_error("batch: cannot allocate %llu bytes of circuit states", (unsigned long long)(state_off * S));
        return SV_ENOMEM;
    }
    if ((rc = dev_upload(b->d_inst, inst, s)) != SV_OK || (rc = dev_upload(b->d_pass, passes, s)) != SV_OK ||
        (rc = dev_upload(b->d_steps, steps, s)) != SV_OK || (rc = dev_upload(b->d_tasks, tasks, s)) != SV_OK ||
        (rc = dev_upload(b->d_z, zs, s)) != SV_OK)
        return rc;
    std::vector<double> zero_part(std::max(1, part_off), 0.0);
    if ((rc = dev_upload(b->d_part, zero_part, s)) != SV_OK)
        return rc;
    std::vector<double> zero_out(std::max(1, out_off), 0.0);
    if ((rc = dev_upload(b->d_out, zero_out, s)) != SV_OK)
        return rc;
    b->nctr = uint32_t(2 + 2 * b->ninst);
    std::vector<uint32_t> zc(b->nctr, 0u);
    if ((rc = dev_upload(b->d_ctr, zc, s)) != SV_OK)
        return rc;
    const size_t mat_bytes = std::max<size_t>(1, b->mat_elems) * 2 * (S / 2);
    if (hipMalloc(&b->d_mats, mat_bytes) != hipSuccess ||
        hipHostMalloc(&b->h_mats, mat_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->h_out, std::max(1, out_off) * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->h_err, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("batch: cannot allocate matrix or output buffers");
        return SV_ENOMEM;
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("batch: upload synchronisation failed");
        return SV_EDEVICE;
    }
    b->lds = batch_lds_bytes(L, S);
    b->grid = batch_grid(b->dtype, b->lds);

    BatchArgs a{};
    a.states = b->d_states;
    a.inst = b->d_inst;
    a.pass = b->d_pass;
    a.steps = b->d_steps;
    a.mats = b->d_mats;
    a.tasks = b->d_tasks;
    a.zmasks = b->d_z;
    a.partials = b->d_part;
    a.out = b->d_out;
    a.ctr = b->d_ctr;
    a.ntasks = b->ntasks;
    a.ninst = uint32_t(b->ninst);
    a.spin_limit = kSpinLimit;
    a.tile_log_max = L;

    // capture: clear counters (kernel, not a memset node), upload matrices,
    // the persistent launch, copy results and the error flag back
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("batch: stream capture could not start");
        return SV_EDEVICE;
    }
    hipError_t e = launch_batch_fill(b->d_ctr, b->nctr, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_mats, b->h_mats, mat_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_batch(b->dtype, a, b->grid, b->lds, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_out, b->d_out, std::max(1, out_off) * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_err, b->d_ctr + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        set_error("batch: graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        return SV_EDEVICE;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        set_error("batch: graph instantiation failed");
        return SV_EDEVICE;
    }
    b->built = true;
    return SV_OK;
}

int run_once(sv_batch *b)
{
    fill_matrices(b);
    *b->h_err = 0;
    if (hipEventRecord(b->ev0, b->stream) != hipSuccess || hipGraphLaunch(b->exec, b->stream) != hipSuccess ||
        hipEventRecord(b->ev1, b->stream) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) {
        set_error("batch: graph launch failed");
        return SV_EDEVICE;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
    b->last_ms = ms;
    if (*b->h_err != 0) {
        set_error("batch: a dependency wait exceeded its spin limit");
        return SV_EDEVICE;
    }
    return SV_OK;
}

bool config_ok(int dtype, const sv_batch_config &c)
{
    const int maxL = dtype == SV_C64 ? 13 : 12;
    return c.tile_bits >= 8 && c.tile_bits <= maxL && c.low_bits >= 0 && c.low_bits <= 4 &&
           c.low_bits <= c.tile_bits - 3 && (c.fuse_width == 1 || c.fuse_width == 2) && c.reserved == 0;
}

int set_gates(sv_batch *b, const sv_gate *const *gates, bool create)
{
    for (int i = 0; i < b->ninst; ++i) {
        const int ng = int(b->gates[i].size());
        for (int k = 0; k < ng; ++k) {
            const sv_gate &g = gates[i][k];
            if (!create) {
                const sv_gate &o = b->gates[i][k];
                bool same = g.kind == o.kind && g.num_targets == o.num_targets && g.num_controls == o.num_controls;
                for (int j = 0; same && j < g.num_targets; ++j)
                    same = g.targets[j] == o.targets[j];
                for (int j = 0; same && j < g.num_controls; ++j)
                    same = g.controls[j] == o.controls[j];
                if (!same) {
                    set_error("batch circuit %d gate %d differs in structure from the created batch", i, k);
                    return SV_EINVAL;
                }
            }
            int rc = validate_gate(g, b->q[i], k);
            if (rc != SV_OK)
                return rc;
            if (!batch_gate_ok(g)) {
                set_error("batch circuit %d gate %d: only one-target gates with <= 1 control or two-target "
                          "matrices are supported", i, k);
                return SV_EUNSUPPORTED;
            }
        }
    }
    for (int i = 0; i < b->ninst; ++i) {
        const int ng = int(b->gates[i].size());
        size_t need = 0;
        for (int k = 0; k < ng; ++k)
            if (gates[i][k].kind == SV_GATE_MATRIX)
                need += size_t(2) << (2 * gates[i][k].num_targets);
        b->matrices[i].resize(need);
        size_t off = 0;
        for (int k = 0; k < ng; ++k) {
            sv_gate g = gates[i][k];
            if (g.kind == SV_GATE_MATRIX) {
                const size_t len = size_t(2) << (2 * g.num_targets);
                std::copy(g.matrix, g.matrix + len, b->matrices[i].begin() + off);
                g.matrix = b->matrices[i].data() + off;
                off += len;
            }
            b->gates[i][k] = g;
        }
    }
    return SV_OK;
}

}  // namespace

extern "C" {

int sv_batch_create(int dtype, int ninst, const int *nqubits, const sv_gate *const *gates, const int *ngates,
                    const uint64_t *const *zmasks, const int *nterms, void *stream, sv_batch_handle *out)
{
    clear_error();
    if (!out || ninst < 1 || !nqubits || !gates || !ngates || !nterms || (dtype != SV_C64 && dtype != SV_C128)) {
        set_error("sv_batch_create: bad arguments");
        return SV_EINVAL;
    }
    sv_batch *b = new (std::nothrow) sv_batch();
    if (!b) {
        set_error("out of host memory");
        return SV_ENOMEM;
    }
    b->dtype = dtype;
    b->ninst = ninst;
    b->q.assign(nqubits, nqubits + ninst);
    b->gates.resize(ninst);
    b->matrices.resize(ninst);
    b->zmasks.resize(ninst);
    for (int i = 0; i < ninst; ++i) {
        if (nqubits[i] < 1 || nqubits[i] > 30 || ngates[i] < 0 || (ngates[i] > 0 && !gates[i]) || nterms[i] < 0 ||
            nterms[i] > kBatchMaxTerms || (nterms[i] > 0 && (!zmasks || !zmasks[i]))) {
            delete b;
            set_error("sv_batch_create: circuit %d has bad size arguments", i);
            return SV_EINVAL;
        }
        b->gates[i].assign(gates[i], gates[i] + ngates[i]);
        for (int t = 0; t < nterms[i]; ++t) {
            if (zmasks[i][t] >> nqubits[i]) {
                delete b;
                set_error("sv_batch_create: circuit %d Z mask %d names a qubit >= %d", i, t, nqubits[i]);
                return SV_EINVAL;
            }
            b->zmasks[i].push_back(zmasks[i][t]);
        }
    }
    int rc = set_gates(b, gates, true);
    if (rc != SV_OK) {
        delete b;
        return rc;
    }
    b->cfg.tile_bits = dtype == SV_C64 ? 13 : 12;
    b->cfg.low_bits = 3;
    b->cfg.fuse_width = 2;
    b->cfg.reserved = 0;
    if (stream) {
        b->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            set_error("sv_batch_create: stream creation failed");
            return SV_EDEVICE;
        }
        b->own_stream = true;
    }
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        sv_batch_destroy(b);
        set_error("sv_batch_create: event creation failed");
        return SV_EDEVICE;
    }
    *out = b;
    return SV_OK;
}

int sv_batch_set_config(sv_batch_handle b, const sv_batch_config *cfg)
{
    clear_error();
    if (!b || !cfg || !config_ok(b->dtype, *cfg)) {
        set_error("sv_batch_set_config: bad configuration");
        return SV_EINVAL;
    }
    if (std::memcmp(cfg, &b->cfg, sizeof *cfg) != 0) {
        b->cfg = *cfg;
        b->built = false;
    }
    return SV_OK;
}

int sv_batch_get_config(sv_batch_handle b, sv_batch_config *cfg)
{
    if (!b || !cfg) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    *cfg = b->cfg;
    return SV_OK;
}

int sv_batch_run(sv_batch_handle b, const sv_gate *const *gates, double *out)
{
    clear_error();
    if (!b || !out) {
        set_error("sv_batch_run: NULL argument");
        return SV_EINVAL;
    }
    int rc;
    if (gates && (rc = set_gates(b, gates, false)) != SV_OK)
        return rc;
    if (!b->built && (rc = build(b)) != SV_OK)
        return rc;
    if ((rc = run_once(b)) != SV_OK)
        return rc;
    std::memcpy(out, b->h_out, size_t(b->total_terms) * sizeof(double));
    return SV_OK;
}

int sv_batch_tune(sv_batch_handle b, int repeats, sv_batch_config *chosen)
{
    clear_error();
    if (!b || repeats < 1) {
        set_error("sv_batch_tune: bad arguments");
        return SV_EINVAL;
    }
    const int maxL = b->dtype == SV_C64 ? 13 : 12;
    sv_batch_config best = b->cfg;
    double best_ms = 1e300;
    for (int L = 11; L <= maxL; ++L)
        for (int low = 2; low <= 4; ++low)
            for (int fw = 1; fw <= 2; ++fw) {
                sv_batch_config c{L, low, fw, 0};
                b->cfg = c;
                b->built = false;
                int rc = build(b);
                if (rc != SV_OK)
                    return rc;
                rc = run_once(b);  // warm-up
                if (rc != SV_OK)
                    return rc;
                double tot = 0.0;
                for (int r = 0; r < repeats; ++r) {
                    if ((rc = run_once(b)) != SV_OK)
                        return rc;
                    tot += b->last_ms;
                }
                if (tot / repeats < best_ms) {
                    best_ms = tot / repeats;
                    best = c;
                }
            }
    b->cfg = best;
    b->built = false;
    int rc = build(b);
    if (rc != SV_OK)
        return rc;
    if (chosen)
        *chosen = best;
    return SV_OK;
}

int sv_batch_last_ms(sv_batch_handle b, double *ms)
{
    if (!b || !ms) {
        set_error("NULL argument");
        return SV_EINVAL;
    }
    *ms = b->last_ms;
    return SV_OK;
}

int sv_batch_destroy(sv_batch_handle b)
{
    if (!b)
        return SV_OK;
    if (b->stream)
        (void)hipStreamSynchronize(b->stream);
    free_build(b);
    if (b->ev0)
        (void)hipEventDestroy(b->ev0);
    if (b->ev1)
        (void)hipEventDestroy(b->ev1);
    if (b->own_stream && b->stream)
        (void)hipStreamDestroy(b->stream);
    delete b;
    return SV_OK;
}

}  // extern "C"
