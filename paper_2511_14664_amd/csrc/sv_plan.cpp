// Host side of the library: its own gate table, gate validation, and the
// fusion planner that groups a gate list into sweeps over the state.
//
// Fusion (paper Sec. 2.1 "State-Vector Simulation"): several gate
// applications are grouped into one operation on the union of their qubits.
// That can raise the flop count, but each sweep over the 2^n amplitudes then
// does more work per byte moved; the widest block worth forming depends on
// the machine and the precision (Sec. 2.1; Sec. 2.2 quotes fusion levels of
// 4-5 qubits on the paper's GPUs).  The planner here is a dependency-aware
// greedy packing into blocks of at most k_max qubits; block matrices are the
// ordered product of their gates, formed in FP64.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <future>

#include "sv_internal.h"

namespace sv {

// ---------------------------------------------------------------------------
// Gate table.  Rotations R_P(t) = exp(-i t P / 2); U3 in the three-angle form
// [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]].
// ---------------------------------------------------------------------------
bool named_gate_matrix(int kind, const double *p, cd out[4])
{
    const cd I(0.0, 1.0);
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (kind) {
    case SV_GATE_H:
        out[0] = r2, out[1] = r2, out[2] = r2, out[3] = -r2;
        return true;
    case SV_GATE_X:
        out[0] = 0.0, out[1] = 1.0, out[2] = 1.0, out[3] = 0.0;
        return true;
    case SV_GATE_Y:
        out[0] = 0.0, out[1] = -I, out[2] = I, out[3] = 0.0;
        return true;
    case SV_GATE_Z:
        out[0] = 1.0, out[1] = 0.0, out[2] = 0.0, out[3] = -1.0;
        return true;
    case SV_GATE_S:
        out[0] = 1.0, out[1] = 0.0, out[2] = 0.0, out[3] = I;
        return true;
    case SV_GATE_T:
        out[0] = 1.0, out[1] = 0.0, out[2] = 0.0, out[3] = std::polar(1.0, M_PI / 4.0);
        return true;
    case SV_GATE_RX: {
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        out[0] = c, out[1] = -I * s, out[2] = -I * s, out[3] = c;
        return true;
    }
    case SV_GATE_RY: {
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        out[0] = c, out[1] = -s, out[2] = s, out[3] = c;
        return true;
    }
    case SV_GATE_RZ:
        out[0] = std::polar(1.0, -0.5 * p[0]), out[1] = 0.0, out[2] = 0.0, out[3] = std::polar(1.0, 0.5 * p[0]);
        return true;
    case SV_GATE_P:
        out[0] = 1.0, out[1] = 0.0, out[2] = 0.0, out[3] = std::polar(1.0, p[0]);
        return true;
    case SV_GATE_U3: {
        const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
        out[0] = c;
        out[1] = -std::polar(1.0, p[2]) * s;
        out[2] = std::polar(1.0, p[1]) * s;
        out[3] = std::polar(1.0, p[1] + p[2]) * c;
        return true;
    }
    default:
        return false;
    }
}

static bool kind_is_diagonal(int kind)
{
    return kind == SV_GATE_Z || kind == SV_GATE_S || kind == SV_GATE_T || kind == SV_GATE_RZ ||
           kind == SV_GATE_P;
}

int validate_gate(const sv_gate &g, int n, int index)
{
    if (g.kind < SV_GATE_H || g.kind > SV_GATE_MATRIX) {
        set_error("gate %d: unknown kind %d", index, g.kind);
        return SV_EINVAL;
    }
    const int k = g.num_targets, c = g.num_controls;
    if (g.kind != SV_GATE_MATRIX && k != 1) {
        set_error("gate %d: named gate kinds take exactly one target (got %d)", index, k);
        return SV_EINVAL;
    }
    if (k < 1 || k > SV_MAX_TARGETS) {
        set_error("gate %d: %d targets (1..%d allowed)", index, k, SV_MAX_TARGETS);
        return SV_EINVAL;
    }
    if (c < 0 || c > SV_MAX_CONTROLS) {
        set_error("gate %d: %d controls (0..%d allowed)", index, c, SV_MAX_CONTROLS);
        return SV_EINVAL;
    }
    if (g.kind == SV_GATE_MATRIX && g.matrix == nullptr) {
        set_error("gate %d: matrix gate with NULL matrix", index);
        return SV_EINVAL;
    }
    uint64_t used = 0;
    for (int j = 0; j < k + c; ++j) {
        const int q = j < k ? g.targets[j] : g.controls[j - k];
        if (q < 0 || q >= n) {
            set_error("gate %d: qubit %d out of range [0, %d)", index, q, n);
            return SV_EINVAL;
        }
        if ((used >> q) & 1) {
            set_error("gate %d: qubit %d used twice", index, q);
            return SV_EINVAL;
        }
        used |= uint64_t(1) << q;
    }
    if (g.kind != SV_GATE_MATRIX) {
        for (int j = 0; j < 3; ++j)
            if (!std::isfinite(g.params[j])) {
                set_error("gate %d: non-finite parameter", index);
                return SV_EINVAL;
            }
    } else {
        const int d = 1 << k;
        for (int j = 0; j < 2 * d * d; ++j)
            if (!std::isfinite(g.matrix[j])) {
                set_error("gate %d: non-finite matrix entry", index);
                return SV_EINVAL;
            }
    }
    return SV_OK;
}

static bool matrix_is_diagonal(const std::vector<cd> &U, int d)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && U[size_t(r) * d + c] != cd(0.0, 0.0))
                return false;
    return true;
}

Block gate_block(const sv_gate &g)
{
    Block b;
    b.k = g.num_targets;
    b.c = g.num_controls;
    for (int j = 0; j < b.k; ++j)
        b.targets[j] = g.targets[j];
    for (int j = 0; j < b.c; ++j)
        b.controls[j] = g.controls[j];
    const int d = 1 << b.k;
    b.U.assign(size_t(d) * d, cd(0.0, 0.0));
    if (g.kind == SV_GATE_MATRIX) {
        for (int j = 0; j < d * d; ++j)
            b.U[j] = cd(g.matrix[2 * j], g.matrix[2 * j + 1]);
        b.diag = matrix_is_diagonal(b.U, d);
    } else {
        cd m[4];
        named_gate_matrix(g.kind, g.params, m);
        for (int j = 0; j < 4; ++j)
            b.U[j] = m[j];
        b.diag = kind_is_diagonal(g.kind);
    }
    b.ngates = 1;
    return b;
}

std::vector<Block> plan_plain(const std::vector<Block> &gates)
{
    return gates;
}

// Left-multiply the d x d matrix M (row-major, split into real and imaginary
// parts) by gate g acting on block positions tpos (targets) and cpos
// (controls): for every row set {base | off_j} (target bits of base zero,
// control bits one) the rows mix through g's matrix.  The row updates run
// across all d columns at once, so the inner loops are unit-stride and
// vectorise; complex products are written out (no library complex calls).
static void left_multiply(double *Mr, double *Mi, int kb, const Block &g, const int *tpos, const int *cpos)
{
    const int d = 1 << kb, kg = g.k, dg = 1 << kg;
    int mt = 0, mc = 0;
    for (int b = 0; b < kg; ++b)
        mt |= 1 << tpos[b];
    for (int j = 0; j < g.c; ++j)
        mc |= 1 << cpos[j];
    int off[64];
    for (int j = 0; j < dg; ++j) {
        off[j] = 0;
        for (int b = 0; b < kg; ++b)
            if ((j >> b) & 1)
                off[j] |= 1 << tpos[b];
    }
    double ur[64 * 64], ui[64 * 64];
    for (int j = 0; j < dg * dg; ++j) {
        ur[j] = g.U[size_t(j)].real();
        ui[j] = g.U[size_t(j)].imag();
    }
    for (int base = 0; base < d; ++base) {
        if ((base & mt) != 0 || (base & mc) != mc)
            continue;
        if (dg == 2) {
            double *r0 = Mr + size_t(base | off[0]) * d, *i0 = Mi + size_t(base | off[0]) * d;
            double *r1 = Mr + size_t(base | off[1]) * d, *i1 = Mi + size_t(base | off[1]) * d;
            for (int c = 0; c < d; ++c) {
                const double ar = r0[c], ai = i0[c], br = r1[c], bi = i1[c];
                r0[c] = (ur[0] * ar - ui[0] * ai) + (ur[1] * br - ui[1] * bi);
                i0[c] = (ur[0] * ai + ui[0] * ar) + (ur[1] * bi + ui[1] * br);
                r1[c] = (ur[2] * ar - ui[2] * ai) + (ur[3] * br - ui[3] * bi);
                i1[c] = (ur[2] * ai + ui[2] * ar) + (ur[3] * bi + ui[3] * br);
            }
            continue;
        }
        if (dg == 4) {
            double *r[4], *im[4];
            for (int j = 0; j < 4; ++j) {
                r[j] = Mr + size_t(base | off[j]) * d;
                im[j] = Mi + size_t(base | off[j]) * d;
            }
            for (int c = 0; c < d; ++c) {
                const double a0 = r[0][c], b0 = im[0][c], a1 = r[1][c], b1 = im[1][c];
                const double a2 = r[2][c], b2 = im[2][c], a3 = r[3][c], b3 = im[3][c];
                for (int q = 0; q < 4; ++q) {
                    const double *xr = ur + 4 * q, *xi = ui + 4 * q;
                    r[q][c] = ((xr[0] * a0 - xi[0] * b0) + (xr[1] * a1 - xi[1] * b1)) +
                              ((xr[2] * a2 - xi[2] * b2) + (xr[3] * a3 - xi[3] * b3));
                    im[q][c] = ((xr[0] * b0 + xi[0] * a0) + (xr[1] * b1 + xi[1] * a1)) +
                               ((xr[2] * b2 + xi[2] * a2) + (xr[3] * b3 + xi[3] * a3));
                }
            }
            continue;
        }
        double *rr[64], *ri[64];
        for (int j = 0; j < dg; ++j) {
            rr[j] = Mr + size_t(base | off[j]) * d;
            ri[j] = Mi + size_t(base | off[j]) * d;
        }
        double vr[64], vi[64];
        for (int c = 0; c < d; ++c) {
            for (int j = 0; j < dg; ++j) {
                vr[j] = rr[j][c];
                vi[j] = ri[j][c];
            }
            for (int r = 0; r < dg; ++r) {
                double sr = 0.0, si = 0.0;
                for (int j = 0; j < dg; ++j) {
                    const double a = ur[r * dg + j], b = ui[r * dg + j];
                    sr += a * vr[j] - b * vi[j];
                    si += a * vi[j] + b * vr[j];
                }
                rr[r][c] = sr;
                ri[r][c] = si;
            }
        }
    }
}

Block fuse(const std::vector<const Block *> &members, uint64_t qmask, bool dense)
{
    if (members.size() == 1 && !dense)
        return *members[0];
    Block out;
    int pos[64];
    int kb = 0;
    for (int q = 0; q < 64; ++q)
        if ((qmask >> q) & 1) {
            out.targets[kb] = q;
            pos[q] = kb++;
        }
    out.k = kb;
    out.c = 0;
    const int d = 1 << kb;
    std::vector<double> Mr(size_t(d) * d, 0.0), Mi(size_t(d) * d, 0.0);  // row-major
    for (int i = 0; i < d; ++i)
        Mr[size_t(i) * d + i] = 1.0;
    bool diag = true;
    int ng = 0;
    for (const Block *g : members) {
        int tpos[SV_MAX_TARGETS], cpos[SV_MAX_CONTROLS];
        for (int b = 0; b < g->k; ++b)
            tpos[b] = pos[g->targets[b]];
        for (int j = 0; j < g->c; ++j)
            cpos[j] = pos[g->controls[j]];
        left_multiply(Mr.data(), Mi.data(), kb, *g, tpos, cpos);
        diag = diag && g->diag;
        ng += g->ngates;
    }
    out.U.resize(size_t(d) * d);
    for (size_t j = 0; j < out.U.size(); ++j)
        out.U[j] = cd(Mr[j], Mi[j]);
    out.diag = diag;
    out.ngates = ng;
    return out;
}

Block densify(const Block &b)
{
    if (b.c == 0)
        return b;
    Block o;
    o.k = b.k + b.c;
    for (int j = 0; j < b.k; ++j)
        o.targets[j] = b.targets[j];
    for (int j = 0; j < b.c; ++j)
        o.targets[b.k + j] = b.controls[j];
    const int d = 1 << o.k, dk = 1 << b.k;
    const int all = ((1 << b.c) - 1) << b.k;  // control bits of the new index
    o.U.assign(size_t(d) * d, cd(0.0, 0.0));
    for (int r = 0; r < d; ++r) {
        if ((r & all) != all) {
            o.U[size_t(r) * d + r] = 1.0;
            continue;
        }
        for (int c = 0; c < d; ++c)
            if ((c & all) == all)
                o.U[size_t(r) * d + c] = b.U[size_t(r & (dk - 1)) * dk + (c & (dk - 1))];
    }
    o.ngates = b.ngates;
    o.diag = b.diag;
    return o;
}

Block group_shape(const std::vector<Block> &gates, const Group &g)
{
    if (g.members.size() == 1)
        return gates[size_t(g.members[0])];
    if (__builtin_popcountll(g.qmask) < 2) {
        std::vector<const Block *> mem;
        for (int i : g.members)
            mem.push_back(&gates[size_t(i)]);
        return fuse(mem, g.qmask);
    }
    Block out;
    for (int q = 0; q < 64; ++q)
        if ((g.qmask >> q) & 1)
            out.targets[out.k++] = q;
    out.diag = true;
    for (int i : g.members) {
        out.diag = out.diag && gates[size_t(i)].diag;
        out.ngates += gates[size_t(i)].ngates;
    }
    return out;
}

uint64_t qubit_mask(const Block &b)
{
    uint64_t m = 0;
    for (int j = 0; j < b.k; ++j)
        m |= uint64_t(1) << b.targets[j];
    for (int j = 0; j < b.c; ++j)
        m |= uint64_t(1) << b.controls[j];
    return m;
}

// Greedy, dependency-aware packing.  Walking the gates in order, a gate joins
// the most recent block among those last touching its qubits when the union
// stays within kmax qubits (it cannot join an earlier one: that block is
// followed by another touching one of the gate's qubits).  A block that
// nothing later touches ("free" block) commutes past everything after it, so
// it may be moved into the block the gate joins when that keeps the union
// within kmax; this packs a layer of one-qubit gates into the entangling
// gates that follow it.
// Second pass over the block sequence: block j joins an earlier block i when
// their union stays within kmax qubits and every block between them acts on
// qubits disjoint from j's (so j commutes back to i); or, symmetrically, i
// joins j when everything between is disjoint from i.  Repeats until no
// merge applies.  dep[] holds each block's qubits for the commutation test,
// g[].qmask those that count towards kmax; at most omax qubits of dep lie
// outside qmask.
static void merge_groups(std::vector<Group> &g, std::vector<uint64_t> &dep, int kmax, int omax, uint64_t freem)
{
    auto popc = [](uint64_t x) { return __builtin_popcountll(x); };
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t i = 0; i < g.size() && !changed; ++i) {
            uint64_t between = 0;  // union of qubits of blocks strictly between i and j
            for (size_t j = i + 1; j < g.size(); ++j) {
                if (popc((g[i].qmask | g[j].qmask) & ~freem) <= kmax &&
                    popc((dep[i] | dep[j]) & ~(g[i].qmask | g[j].qmask)) <= omax) {
                    if ((between & dep[j]) == 0) {
                        // move j back into i: members of j follow those of i
                        g[i].members.insert(g[i].members.end(), g[j].members.begin(), g[j].members.end());
                        g[i].qmask |= g[j].qmask;
                        dep[i] |= dep[j];
                        g.erase(g.begin() + long(j));
                        dep.erase(dep.begin() + long(j));
                        changed = true;
                        break;
                    }
                    if ((between & dep[i]) == 0) {
                        // move i forward into j: members of i precede those of j
                        g[j].members.insert(g[j].members.begin(), g[i].members.begin(), g[i].members.end());
                        g[j].qmask |= g[i].qmask;
                        dep[j] |= dep[i];
                        g.erase(g.begin() + long(i));
                        dep.erase(dep.begin() + long(i));
                        changed = true;
                        break;
                    }
                }
                between |= dep[j];
                if (popc(between | dep[i]) > 64)
                    break;
            }
        }
    }
}

// The greedy packing over items with qubit masks dep (every qubit the item
// touches: ordering) and budget masks (the qubits that count towards kmax).
// With dep == budget this is the plain greedy plan.  Pass planning gives a
// diagonal gate a second, smaller budget mask (qubits outside a pass tile are
// constant per tile, so there a diagonal gate needs only its in-tile qubits):
// a gate joins with its full mask when that fits, else with the small one,
// and a block may hold at most omax qubits outside its budget.  Qubits in
// freem do not count towards kmax (a pass tile holds the lowest index bits
// whether or not its gates act on them).
static std::vector<Group> greedy_masks(const std::vector<uint64_t> &depm, const std::vector<uint64_t> &budm,
                                       const std::vector<uint64_t> *minm, int kmax, int omax,
                                       std::vector<uint64_t> *dep_out, uint64_t freem = 0)
{
    // blocks as linked member lists (head, tail, next[]): moving a free
    // block into another splices its list in front in constant time
    struct PB {
        int head = -1, tail = -1, size = 0;
        uint64_t qmask = 0, dep = 0;
        bool alive = true;
    };
    const int N = int(depm.size());
    std::vector<PB> pb;
    pb.reserve(size_t(N));
    std::vector<int> next(size_t(N), -1);
    int last[64];
    std::fill(last, last + 64, -1);
    auto popc = [](uint64_t x) { return __builtin_popcountll(x); };
    auto fits = [&](uint64_t bud, uint64_t dep) {
        return popc(bud & ~freem) <= kmax && popc(dep & ~bud) <= omax;
    };
    // set bits of a mask, lowest first
    auto each_bit = [](uint64_t x, auto &&f) {
        while (x) {
            f(__builtin_ctzll(x));
            x &= x - 1;
        }
    };
    for (int i = 0; i < N; ++i) {
        const uint64_t gm = depm[size_t(i)];
        uint64_t gb = budm[size_t(i)];
        int cand = -1;
        each_bit(gm, [&](int q) { cand = std::max(cand, last[q]); });
        int target = -1;
        if (cand >= 0) {
            if (fits(pb[cand].qmask | gb, pb[cand].dep | gm)) {
                target = cand;
            } else if (minm && fits(pb[cand].qmask | (*minm)[size_t(i)], pb[cand].dep | gm)) {
                gb = (*minm)[size_t(i)];
                target = cand;
            }
        }
        if (target < 0) {
            if (!fits(gb, gm) && minm && fits((*minm)[size_t(i)], gm))
                gb = (*minm)[size_t(i)];
            pb.push_back(PB());
            target = int(pb.size()) - 1;
        }
        if (fits(gb, gm)) {
            each_bit(gm, [&](int q) {
                const int b = last[q];
                if (b < 0 || b == target || !pb[b].alive)
                    return;
                bool movable = true;
                each_bit(pb[b].dep, [&](int r) { movable = movable && last[r] == b; });
                if (!movable || !fits(pb[target].qmask | pb[b].qmask | gb, pb[target].dep | pb[b].dep | gm))
                    return;
                // the members of b go before those of target
                PB &t = pb[target], &f = pb[b];
                if (f.head >= 0) {
                    if (t.head >= 0)
                        next[size_t(f.tail)] = t.head;
                    else
                        t.tail = f.tail;
                    t.head = f.head;
                    t.size += f.size;
                }
                t.qmask |= f.qmask;
                t.dep |= f.dep;
                f.alive = false;
                f.head = f.tail = -1;
                f.size = 0;
                each_bit(f.dep, [&](int r) { last[r] = target; });
            });
        }
        PB &t = pb[target];
        if (t.tail >= 0)
            next[size_t(t.tail)] = i;
        else
            t.head = i;
        t.tail = i;
        ++t.size;
        t.qmask |= gb;
        t.dep |= gm;
        each_bit(gm, [&](int q) { last[q] = target; });
    }
    std::vector<Group> out;
    std::vector<uint64_t> dep;
    for (const PB &b : pb) {
        if (!b.alive || b.size == 0)
            continue;
        Group g{std::vector<int>(), b.qmask};
        g.members.reserve(size_t(b.size));
        for (int x = b.head; x >= 0; x = next[size_t(x)])
            g.members.push_back(x);
        out.push_back(std::move(g));
        dep.push_back(b.dep);
    }
    merge_groups(out, dep, kmax, omax, freem);
    if (dep_out)
        *dep_out = dep;
    return out;
}

std::vector<Group> group_greedy(const std::vector<Block> &gates, int kmax)
{
    std::vector<uint64_t> m(gates.size());
    for (size_t i = 0; i < gates.size(); ++i)
        m[i] = qubit_mask(gates[i]);
    return greedy_masks(m, m, nullptr, kmax, 64, nullptr);
}

// A diagonal gate whose entries all have modulus 1 (to rounding) is a pure
// phase on each basis state, so a pass may fold it in as angles; a diagonal
// with other moduli (not unitary) keeps its magnitudes by taking the
// ordinary block path.
bool is_phase_gate(const Block &b)
{
    if (!b.diag || b.k + b.c > kMaxPhaseQubits)
        return false;
    const int d = 1 << b.k;
    for (int x = 0; x < d; ++x)
        if (std::fabs(std::norm(b.U[size_t(x) * d + x]) - 1.0) > 1e-10)
            return false;
    return true;
}

uint64_t outer_capable(const Block &b)
{
    if (is_phase_gate(b))
        return qubit_mask(b);
    uint64_t m = 0;
    for (int j = 0; j < b.c; ++j)
        m |= uint64_t(1) << b.controls[j];
    return m;
}

// Qubits a gate acts on non-diagonally (the targets of a non-diagonal matrix;
// controls and diagonal matrices only multiply by phases).
static uint64_t nondiag_mask(const Block &b)
{
    if (b.diag)
        return 0;
    uint64_t m = 0;
    for (int j = 0; j < b.k; ++j)
        m |= uint64_t(1) << b.targets[j];
    return m;
}

// Sub-blocks of one kernel pass.  Gates whose qubits all lie in the pass
// tile are packed greedily into <= 4-qubit blocks; a diagonal gate with
// qubits outside the tile takes part through its in-tile qubits only.  If a
// block's gates reach at most kMaxVariantBits qubits outside the tile, the
// block keeps all its gates in order and is staged once per value of those
// qubits.  Otherwise each such gate is attached to its block as a phase
// applied before the block's matrix (front: it commutes with every member
// before it) or after it (back: it commutes with every member after it), and
// the block is split where neither holds.
// Candidate partitions of one pass's gates (items with qubit masks dep and
// budget masks bud, in circuit order) into blocks of <= 4 tile qubits: the
// greedy packing over several gate orders.  Items touching a common qubit
// keep their relative order in every order tried, so each partition is the
// circuit's product: the order given, its reverse (the blocks of a partition
// valid for the reversed list, taken in reverse with their members in
// reverse, are a valid partition of the list), and `trials` seeded random
// orders consistent with the dependencies.  A block lists its items
// in an order consistent with the dependencies (not necessarily ascending).
static std::vector<std::vector<Group>> pass_partitions(const std::vector<uint64_t> &dep,
                                                       const std::vector<uint64_t> &bud, int trials)
{
    const int m = int(dep.size());
    std::vector<std::vector<Group>> out;
    out.push_back(greedy_masks(dep, bud, nullptr, 4, 64, nullptr));
    auto add = [&](const std::vector<int> &order, bool reversed) {
        std::vector<uint64_t> d(static_cast<size_t>(m)), b(static_cast<size_t>(m));
        for (int i = 0; i < m; ++i) {
            d[size_t(i)] = dep[size_t(order[size_t(i)])];
            b[size_t(i)] = bud[size_t(order[size_t(i)])];
        }
        std::vector<Group> g = greedy_masks(d, b, nullptr, 4, 64, nullptr);
        for (Group &x : g)
            for (int &i : x.members)
                i = order[size_t(i)];
        if (reversed) {
            std::reverse(g.begin(), g.end());
            for (Group &x : g)
                std::reverse(x.members.begin(), x.members.end());
        }
        out.push_back(std::move(g));
    };
    std::vector<int> order(static_cast<size_t>(m));
    for (int i = 0; i < m; ++i)
        order[size_t(i)] = m - 1 - i;
    add(order, true);
    // random linear extensions: repeatedly take a random item whose
    // predecessors (earlier items sharing a qubit) are all taken
    if (trials <= 0)
        return out;
    uint64_t rng = 0x9E3779B97F4A7C15ull ^ uint64_t(m);
    std::vector<int> npred(static_cast<size_t>(m));
    std::vector<int> ready;
    for (int trial = 0; trial < trials; ++trial) {
        for (int i = 0; i < m; ++i) {
            int c = 0;
            for (int j = 0; j < i; ++j)
                if (dep[size_t(j)] & dep[size_t(i)])
                    ++c;
            npred[size_t(i)] = c;
        }
        ready.clear();
        for (int i = 0; i < m; ++i)
            if (npred[size_t(i)] == 0)
                ready.push_back(i);
        order.clear();
        while (!ready.empty()) {
            rng ^= rng << 13;
            rng ^= rng >> 7;
            rng ^= rng << 17;
            const size_t pick = size_t(rng % ready.size());
            const int i = ready[pick];
            ready[pick] = ready.back();
            ready.pop_back();
            order.push_back(i);
            for (int j = i + 1; j < m; ++j)
                if ((dep[size_t(i)] & dep[size_t(j)]) && --npred[size_t(j)] == 0)
                    ready.push_back(j);
        }
        add(order, false);
    }
    return out;
}

// The pass's blocks from one partition of its gates (sub: groups of
// indices into members).
static void pass_subblocks_from(const std::vector<Block> &gates, const std::vector<int> &members, uint64_t tmask,
                                const std::vector<uint64_t> &depm, const std::vector<char> &phase,
                                const std::vector<Group> &sub, PassGroup &w)
{
    w.subs.clear();
    w.front.clear();
    w.back.clear();
    w.vq.clear();
    for (const Group &sg : sub) {
        // few outer qubits: one matrix per value of them, gates kept in order
        uint64_t outer = 0;
        for (int i : sg.members)
            outer |= qubit_mask(gates[size_t(members[size_t(i)])]) & ~tmask;
        if (__builtin_popcountll(outer) <= kMaxVariantBits) {
            std::vector<int> all;
            for (int i : sg.members)
                all.push_back(members[size_t(i)]);
            w.subs.push_back(Group{std::move(all), sg.qmask});
            w.front.emplace_back();
            w.back.emplace_back();
            w.vq.push_back(outer);
            continue;
        }
        bool nondiag_outer = false;
        for (int i : sg.members)
            if (phase[size_t(i)] && !is_phase_gate(gates[size_t(members[size_t(i)])]))
                nondiag_outer = true;
        if (nondiag_outer) {
            // a gate other than a phase gate, with controls outside the
            // tile, has no phase form: split into consecutive parts of
            // <= kMaxVariantBits outer qubits, each staged with variants
            std::vector<int> part;
            uint64_t pq = 0, po = 0;
            for (int i : sg.members) {
                const uint64_t qm = qubit_mask(gates[size_t(members[size_t(i)])]);
                if (!part.empty() && __builtin_popcountll(po | (qm & ~tmask)) > kMaxVariantBits) {
                    w.subs.push_back(Group{part, pq});
                    w.front.push_back({});
                    w.back.push_back({});
                    w.vq.push_back(po);
                    part.clear();
                    pq = po = 0;
                }
                part.push_back(members[size_t(i)]);
                pq |= depm[size_t(i)];
                po |= qm & ~tmask;
            }
            w.subs.push_back(Group{part, pq});
            w.front.push_back({});
            w.back.push_back({});
            w.vq.push_back(po);
            continue;
        }
        // sg.members index `members`; walk them in order, splitting where a
        // phase commutes neither to the front nor to the back
        std::vector<int> reg, fr, bk;
        uint64_t qm = 0;
        auto flush = [&]() {
            if (reg.empty() && fr.empty() && bk.empty())
                return;
            w.subs.push_back(Group{std::move(reg), qm});
            w.front.push_back(std::move(fr));
            w.back.push_back(std::move(bk));
            w.vq.push_back(0);
            reg.clear();
            fr.clear();
            bk.clear();
            qm = 0;
        };
        const size_t m = sg.members.size();
        for (size_t a = 0; a < m; ++a) {
            const size_t i = size_t(sg.members[a]);
            const int gi = members[i];
            if (!phase[i]) {
                reg.push_back(gi);
                qm |= depm[i];
                continue;
            }
            const uint64_t in = depm[i];
            uint64_t before = 0, after = 0;
            for (int r : reg)
                before |= nondiag_mask(gates[size_t(r)]);
            for (size_t b2 = a + 1; b2 < m; ++b2)
                if (!phase[size_t(sg.members[b2])])
                    after |= nondiag_mask(gates[size_t(members[size_t(sg.members[b2])])]);
            if ((before & in) == 0) {
                fr.push_back(gi);
            } else if ((after & in) == 0) {
                bk.push_back(gi);
            } else {
                flush();
                fr.push_back(gi);
            }
            qm |= in;
        }
        flush();
    }
}

// A pass's blocks: of the candidate partitions of its gates, the one whose
// blocks cost least in the pass model (0.22 per block, 0.31 per block with
// phase terms); the first candidate (circuit order) wins ties.
static void pass_subblocks(const std::vector<Block> &gates, const std::vector<int> &members, uint64_t tmask,
                           int trials, PassGroup &w)
{
    std::vector<uint64_t> depm(members.size());
    std::vector<char> phase(members.size(), 0);
    for (size_t i = 0; i < members.size(); ++i) {
        const uint64_t qm = qubit_mask(gates[size_t(members[i])]);
        phase[i] = (qm & ~tmask) != 0;  // phase gates, or controls, outside the tile
        depm[i] = qm & tmask;
    }
    auto cost = [](const PassGroup &p) {
        double c = 0;
        for (size_t i = 0; i < p.subs.size(); ++i)
            c += (p.front[i].empty() && p.back[i].empty()) ? 0.22 : 0.31;
        return c;
    };
    double best = 0;
    bool have = false;
    PassGroup tmp;
    for (const std::vector<Group> &sub : pass_partitions(depm, depm, trials)) {
        pass_subblocks_from(gates, members, tmask, depm, phase, sub, tmp);
        const double c = cost(tmp);
        if (!have || c < best - 1e-9) {
            best = c;
            have = true;
            w.subs.swap(tmp.subs);
            w.front.swap(tmp.front);
            w.back.swap(tmp.back);
            w.vq.swap(tmp.vq);
        }
    }
}

std::vector<Block> prefuse_diagonal_pairs(const std::vector<Block> &gates)
{
    const size_t N = gates.size();
    std::vector<char> used(N, 0);
    std::vector<uint64_t> qm(N);
    for (size_t i = 0; i < N; ++i)
        qm[i] = qubit_mask(gates[i]);
    std::vector<Block> out;
    out.reserve(N);
    std::vector<size_t> idx;
    for (size_t i = 0; i < N; ++i) {
        if (used[i])
            continue;
        const Block &g = gates[i];
        const uint64_t pair = qm[i];
        if (g.diag || __builtin_popcountll(pair) != 2) {
            out.push_back(g);
            continue;
        }
        // gates after i on the pair's qubits, up to the first that also
        // touches another qubit; gates on other qubits commute past the run.
        // The run's 4x4 product grows one gate at a time (the same products
        // in the same order as fusing the whole run afresh).
        int pos[64], tpos[SV_MAX_TARGETS], cpos[SV_MAX_CONTROLS];
        pos[__builtin_ctzll(pair)] = 0;
        pos[63 - __builtin_clzll(pair)] = 1;
        double Mr[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1}, Mi[16] = {};
        auto mul = [&](const Block &x) {
            for (int b = 0; b < x.k; ++b)
                tpos[b] = pos[x.targets[b]];
            for (int j = 0; j < x.c; ++j)
                cpos[j] = pos[x.controls[j]];
            left_multiply(Mr, Mi, 2, x, tpos, cpos);
        };
        mul(g);
        idx.clear();
        bool fused = false;
        for (size_t j = i + 1; j < N && idx.size() < 15; ++j) {
            if (used[j])
                continue;
            const uint64_t m = qm[j];
            if ((m & pair) == 0)
                continue;
            if ((m & ~pair) != 0)
                break;
            idx.push_back(j);
            mul(gates[j]);
            bool diag = true;
            for (int r = 0; r < 4 && diag; ++r)
                for (int c = 0; c < 4; ++c)
                    if (r != c && (Mr[r * 4 + c] != 0.0 || Mi[r * 4 + c] != 0.0)) {
                        diag = false;
                        break;
                    }
            if (diag) {
                Block f;
                f.k = 2;
                f.c = 0;
                f.targets[0] = __builtin_ctzll(pair);
                f.targets[1] = 63 - __builtin_clzll(pair);
                f.U.resize(16);
                for (int e = 0; e < 16; ++e)
                    f.U[size_t(e)] = cd(Mr[e], Mi[e]);
                f.diag = true;
                f.ngates = g.ngates;
                for (size_t x : idx) {
                    f.ngates += gates[x].ngates;
                    used[x] = 1;
                }
                out.push_back(std::move(f));
                fused = true;
                break;
            }
        }
        if (!fused)
            out.push_back(g);
    }
    return out;
}

// One pass plan.  phases: 0 = phase gates count all their qubits (no outer
// qubits); 1 = all their qubits when that fits, else only those at low
// physical positions; 2 = only those at low physical positions.
static std::vector<PassGroup> pass_plan(const std::vector<Block> &gates, int pass_qubits, int max_fused, int n,
                                        int T0, const int *phys, int phases, int trials)
{
    std::vector<uint64_t> depm(gates.size()), minm(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) {
        const Block &g = gates[i];
        depm[i] = minm[i] = qubit_mask(g);
        const uint64_t cap = phases > 0 ? outer_capable(g) : 0;
        if (cap) {
            uint64_t low = 0;
            for (int q = 0; q < 64; ++q)
                if (((cap >> q) & 1) && (phys ? phys[q] : q) < kPassLowBits)
                    low |= uint64_t(1) << q;
            minm[i] = (depm[i] & ~cap) | low;
        }
    }
    std::vector<uint64_t> pdep;
    // a pass keeps at least T0 index bits off its outer qubits for the tile
    const int omax = std::max(0, n - T0);
    // the tile always holds the T0 - kMaxPassQubits lowest index bits (its
    // contiguous runs), so qubits there join a pass without using its budget
    uint64_t freem = 0;
    for (int q = 0; q < n; ++q)
        if ((phys ? phys[q] : q) < T0 - kMaxPassQubits)
            freem |= uint64_t(1) << q;
    const std::vector<Group> pg = phases == 2 ? greedy_masks(depm, minm, nullptr, pass_qubits, omax, &pdep, freem)
                                              : greedy_masks(depm, depm, &minm, pass_qubits, omax, &pdep, freem);
    std::vector<PassGroup> out(pg.size());
    std::vector<Block> mem;
    for (size_t i = 0; i < pg.size(); ++i) {
        PassGroup &w = out[i];
        w.qmask = pg[i].qmask;
        w.omask = pdep[i] & ~pg[i].qmask;
        for (int m : pg[i].members)
            w.ngates += gates[size_t(m)].ngates;
        const int q = __builtin_popcountll(w.qmask), o = __builtin_popcountll(w.omask);
        const int qb = __builtin_popcountll(w.qmask & ~freem);
        w.kernel = n >= T0 && q >= 1 && qb <= kMaxPassQubits && q <= T0 && n - o >= T0;
        if (w.kernel) {
            pass_subblocks(gates, pg[i].members, w.qmask, trials, w);
            int term_blocks = 0;
            for (size_t j = 0; j < w.subs.size(); ++j) {
                if (__builtin_popcountll(w.subs[j].qmask) > 4)
                    w.kernel = false;
                term_blocks += !w.front[j].empty() || !w.back[j].empty();
            }
            if (term_blocks > kMaxTermBlocks)
                w.kernel = false;
        }
        if (!w.kernel) {
            // ordinary sweeps over the pass's gates (all qubits count)
            mem.clear();
            for (int m : pg[i].members)
                mem.push_back(gates[size_t(m)]);
            std::vector<Group> g = group_greedy(mem, max_fused);
            for (Group &x : g)
                for (int &m : x.members)
                    m = pg[i].members[size_t(m)];
            w.subs = g;
            w.front.assign(g.size(), {});
            w.back.assign(g.size(), {});
            w.vq.assign(g.size(), 0);
            w.qmask = pdep[i];
            w.omask = 0;
        }
    }
    return out;
}

// Relative time of a pass plan in units of one HBM round trip of the state:
// a kernel pass costs max(1, 0.53 + 0.22 nsub) (the matrix cores bind from
// three blocks on: measured slope and intercept of the pass kernel on
// MI355X, the same in both precisions to within a few percent); a block
// carrying per-tile phase terms costs 0.31 instead of 0.22 (measured); a
// sweep costs 1.
double pass_plan_cost(const std::vector<PassGroup> &plan)
{
    double c = 0.0;
    for (const PassGroup &w : plan) {
        if (!w.kernel) {
            c += double(w.subs.size());
            continue;
        }
        double b = 0.53;
        for (size_t i = 0; i < w.subs.size(); ++i)
            b += (w.front[i].empty() && w.back[i].empty()) ? 0.22 : 0.31;
        c += std::max(1.0, b);
    }
    return c;
}

std::vector<std::vector<PassGroup>> pass_plan_candidates(const std::vector<Block> &gates, int pass_qubits,
                                                         int max_fused, int n, int T0, const int *phys, int orders)
{
    std::vector<std::vector<PassGroup>> cands;
    // Three candidate plans, each pass's gates partitioned in circuit order
    // and in reverse; the cheapest is then re-partitioned over random gate
    // orders as well, and re-planned over random orders of the whole
    // circuit.  By default only when the state is large enough for a pass
    // (~13 ms at 32 qubits) to outweigh the host time of the search (tens of
    // ms on a few thousand gates).
    constexpr int kSearchQubits = 32, kDefaultOrders = 16;
    const int trials = orders > 0 ? std::min(orders, kMaxPassOrders)
                                  : (orders == 0 && n >= kSearchQubits ? kDefaultOrders : 0);
    bool any_phase = false;
    for (const Block &g : gates)
        any_phase = any_phase || outer_capable(g) != 0;
    // the candidates are independent: the two with outer qubits are planned
    // on worker threads while this thread plans the first (they sit on the
    // critical path of every circuit applied)
    std::future<std::vector<PassGroup>> alt[2];
    for (int ph = 1; ph <= 2 && any_phase; ++ph)
        alt[ph - 1] = std::async(std::launch::async, [&, ph]() {
            return pass_plan(gates, pass_qubits, max_fused, n, T0, phys, ph, 0);
        });
    cands.push_back(pass_plan(gates, pass_qubits, max_fused, n, T0, phys, 0, 0));
    double cbest = pass_plan_cost(cands.back());
    int pbest = 0;
    for (int ph = 1; ph <= 2 && any_phase; ++ph) {
        cands.push_back(alt[ph - 1].get());
        const double c = pass_plan_cost(cands.back());
        if (c < cbest) {
            cbest = c;
            pbest = ph;
        }
    }
    if (trials > 0) {
        // The same plan over seeded random gate orders of the whole circuit
        // (gates sharing a qubit keep their order; the others commute): the
        // pass grouping sees other gates side by side.  One task per order,
        // each with its own seed, so the result does not depend on their
        // timing; ties go to the earlier candidate.
        const size_t m = gates.size();
        std::vector<int> succ_head(m, -1), succ_next, succ_to;
        {
            int last[64];
            std::fill(last, last + 64, -1);
            for (size_t i = 0; i < m; ++i) {
                uint64_t x = qubit_mask(gates[i]);
                int preds[64], np = 0;
                while (x) {
                    const int q = __builtin_ctzll(x);
                    x &= x - 1;
                    if (last[q] >= 0 && std::find(preds, preds + np, last[q]) == preds + np)
                        preds[np++] = last[q];
                    last[q] = int(i);
                }
                for (int k = 0; k < np; ++k) {
                    succ_next.push_back(succ_head[size_t(preds[k])]);
                    succ_to.push_back(int(i));
                    succ_head[size_t(preds[k])] = int(succ_to.size()) - 1;
                }
            }
        }
        auto plan_order = [&](int trial) {
            uint64_t rng = 0xD1B54A32D192ED03ull ^ (uint64_t(m) << 8) ^ uint64_t(trial + 1) * 0x9E3779B97F4A7C15ull;
            std::vector<int> npred(m, 0), order, ready;
            for (int to : succ_to)
                ++npred[size_t(to)];
            for (size_t i = 0; i < m; ++i)
                if (npred[i] == 0)
                    ready.push_back(int(i));
            while (!ready.empty()) {
                rng ^= rng << 13;
                rng ^= rng >> 7;
                rng ^= rng << 17;
                const size_t pick = size_t(rng % ready.size());
                const int i = ready[pick];
                ready[pick] = ready.back();
                ready.pop_back();
                order.push_back(i);
                for (int e = succ_head[size_t(i)]; e >= 0; e = succ_next[size_t(e)])
                    if (--npred[size_t(succ_to[size_t(e)])] == 0)
                        ready.push_back(succ_to[size_t(e)]);
            }
            std::vector<Block> pg(m);
            for (size_t i = 0; i < m; ++i)
                pg[i] = gates[size_t(order[i])];
            std::vector<PassGroup> q = pass_plan(pg, pass_qubits, max_fused, n, T0, phys, pbest, trials);
            for (PassGroup &w : q) {
                for (Group &g : w.subs)
                    for (int &x : g.members)
                        x = order[size_t(x)];
                for (auto &f : w.front)
                    for (int &x : f)
                        x = order[size_t(x)];
                for (auto &b : w.back)
                    for (int &x : b)
                        x = order[size_t(x)];
            }
            return q;
        };
        std::vector<std::future<std::vector<PassGroup>>> fut;
        for (int trial = 0; trial < trials; ++trial)
            fut.push_back(std::async(std::launch::async, plan_order, trial));
        // meanwhile: the winner in circuit order, each pass split over random
        // orders of its own gates
        cands.push_back(pass_plan(gates, pass_qubits, max_fused, n, T0, phys, pbest, trials));
        for (auto &f : fut)
            cands.push_back(f.get());
    }
    return cands;
}

std::vector<PassGroup> plan_passes(const std::vector<Block> &gates, int pass_qubits, int max_fused, int n, int T0,
                                   const int *phys, int orders)
{
    // the cheapest candidate in the pass model; the earliest wins ties
    std::vector<std::vector<PassGroup>> cands =
        pass_plan_candidates(gates, pass_qubits, max_fused, n, T0, phys, orders);
    size_t best = 0;
    double cbest = pass_plan_cost(cands[0]);
    for (size_t i = 1; i < cands.size(); ++i) {
        const double c = pass_plan_cost(cands[i]);
        if (c < cbest) {
            cbest = c;
            best = i;
        }
    }
    return std::move(cands[best]);
}

std::vector<Block> plan_greedy(const std::vector<Block> &gates, int kmax)
{
    std::vector<Block> out;
    for (const Group &g : group_greedy(gates, kmax)) {
        std::vector<const Block *> mem;
        for (int i : g.members)
            mem.push_back(&gates[i]);
        out.push_back(fuse(mem, g.qmask));
    }
    return out;
}

int plan_circuit(int n, int dtype, const sv_gate *gates, int ngates, const sv_plan_opts &o,
                 std::vector<Block> &out)
{
    (void)dtype;
    if (ngates < 0 || (ngates > 0 && gates == nullptr)) {
        set_error("bad gate list");
        return SV_EINVAL;
    }
    if (o.mode == SV_PLAN_PASSES) {
        set_error("pass plans (SV_PLAN_PASSES) run through sv_apply_circuit only");
        return SV_EINVAL;
    }
    if (o.mode < SV_PLAN_PLAIN || o.mode > SV_PLAN_LEARNED) {
        set_error("unknown plan mode %d", o.mode);
        return SV_EINVAL;
    }
    if (o.pass_qubits != 0 || o.pass_orders != 0 || o.pass_tile != 0) {
        set_error("pass_qubits, pass_orders and pass_tile must be 0 outside SV_PLAN_PASSES");
        return SV_EINVAL;
    }
    if (o.mode != SV_PLAN_PLAIN && (o.max_fused < 1 || o.max_fused > SV_MAX_TARGETS)) {
        set_error("max_fused %d outside 1..%d", o.max_fused, SV_MAX_TARGETS);
        return SV_EINVAL;
    }
    if (o.precision != SV_PREC_NATIVE && o.precision != SV_PREC_BF16X3 && o.precision != SV_PREC_BF16X6) {
        set_error("unknown precision mode %d", o.precision);
        return SV_EINVAL;
    }
    std::vector<Block> blocks;
    blocks.reserve(size_t(ngates));
    for (int i = 0; i < ngates; ++i) {
        int rc = validate_gate(gates[i], n, i);
        if (rc != SV_OK)
            return rc;
        blocks.push_back(gate_block(gates[i]));
    }
    if (o.mode == SV_PLAN_PLAIN)
        out = plan_plain(blocks);
    else
        out = plan_greedy(blocks, o.max_fused);
    return SV_OK;
}

double block_bytes(int n, int dtype, const Block &b, const int *phys_t, const int *phys_c)
{
    const double S = dtype == SV_C64 ? 8.0 : 16.0;
    // bits below log2(128 / S) share 128-byte lines with untouched amplitudes
    const int line_bits = dtype == SV_C64 ? 4 : 3;
    int fixed_hi = 0;
    for (int j = 0; j < b.c; ++j)
        if (phys_c[j] >= line_bits)
            ++fixed_hi;
    if (b.k == 1 && b.diag && b.U[0] == cd(1.0, 0.0) && phys_t[0] >= line_bits)
        ++fixed_hi;
    return 2.0 * S * std::ldexp(1.0, n - fixed_hi);
}

double block_flops(int n, const Block &b)
{
    const double touched = std::ldexp(1.0, n - b.c);
    if (b.k == 1 && b.diag) {
        const double t = (b.U[0] == cd(1.0, 0.0)) ? touched / 2 : touched;
        return 6.0 * t;
    }
    return (8.0 * double(1 << b.k) - 2.0) * touched;
}

}  // namespace sv
