// Internal declarations of the state-vector library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "sv.h"

namespace sv {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

// ---------------------------------------------------------------------------
// Host-side operation descriptions
// ---------------------------------------------------------------------------

// One sweep over the state: a dense 2^k x 2^k matrix on `targets` (logical
// qubits), applied where all `controls` are 1.  `diag` marks a diagonal matrix.
struct Block {
    int k = 0;
    int targets[SV_MAX_TARGETS] = {};
    int c = 0;
    int controls[SV_MAX_CONTROLS] = {};
    std::vector<cd> U;   // 2^k x 2^k row-major, bit b of the index = targets[b]
    int ngates = 0;      // input gates folded into this block
    bool diag = false;
};

// Gate table of the library: 2x2 matrix of a named one-qubit kind.
bool named_gate_matrix(int kind, const double *params, cd out[4]);

// Validate a gate against an n-qubit register; returns SV_OK or SV_EINVAL
// (message set).
int validate_gate(const sv_gate &g, int n, int index);

// Turn a validated gate into an unfused block.
Block gate_block(const sv_gate &g);

// Plans
int plan_circuit(int n, int dtype, const sv_gate *gates, int ngates, const sv_plan_opts &o,
                 std::vector<Block> &out);
std::vector<Block> plan_plain(const std::vector<Block> &gates);
std::vector<Block> plan_greedy(const std::vector<Block> &gates, int kmax);

// Structure of a greedy plan: member gate indices (in application order) and
// the union of their qubits, per block.
struct Group {
    std::vector<int> members;
    uint64_t qmask;
};
std::vector<Group> group_greedy(const std::vector<Block> &gates, int kmax);
// Fuse gates into one block on the qubits of qmask (targets ascending); a
// single member is returned unchanged unless dense is set.
Block fuse(const std::vector<const Block *> &members, uint64_t qmask, bool dense = false);
// Diagonal gates of at most this many qubits (targets + controls) may act on
// qubits outside a pass tile, as per-tile phases ("phase gates").
constexpr int kMaxPhaseQubits = 4;
// Physical index bits below this are tile bits of every pass: a phase gate's
// qubits there count towards the pass budget.
constexpr int kPassLowBits = 6;
// A pass block whose phase gates reach at most this many qubits outside the
// tile is staged as one fused matrix per value of those index bits.
constexpr int kMaxVariantBits = 4;
bool is_phase_gate(const Block &b);
// Qubits of a gate that may lie outside a pass tile: every qubit of a phase
// gate, the controls of any other gate (per tile it is then the gate or the
// identity).
uint64_t outer_capable(const Block &b);
// One pass of an SV_PLAN_PASSES plan: the greedy groups of the circuit with a
// pass_qubits budget on their tile qubits (qmask); phase gates may also touch
// qubits outside the tile (omask), which are constant within each tile.  A
// kernel pass is sub-grouped into <= 4-qubit blocks: subs[i].members are the
// gates fused into block i's matrix, front[i] / back[i] the phase gates with
// qubits outside the tile applied just before / after it.  Otherwise (a
// wider gate, or the state below the pass tile) subs are <= max_fused-qubit
// sweeps over all the pass's gates.  Member indices refer to the circuit's
// gate list.  A block with variant qubits vq[i] (outer qubits of its phase
// gates, at most kMaxVariantBits) instead holds every gate in members, phase
// gates included, and is staged as one matrix per value of those qubits.
struct PassGroup {
    bool kernel = false;
    uint64_t qmask = 0;
    uint64_t omask = 0;
    std::vector<Group> subs;
    std::vector<std::vector<int>> front, back;
    std::vector<uint64_t> vq;
    int ngates = 0;
    int tile_log = 0;  // kernel pass: LDS tile width chosen by the planner (0: by its blocks)
};
// Runs of gates on one qubit pair whose product is diagonal (CX RZ CX =
// exp(-i theta/2 Z Z)) become one phase gate, placed at the run's first gate
// (the gates skipped over act on other qubits and commute with the run), so
// that pass planning may keep one of the pair outside the tile.
std::vector<Block> prefuse_diagonal_pairs(const std::vector<Block> &gates);
// phys: logical -> physical qubit map (nullptr: identity); T0: smallest pass
// tile (log2 amplitudes) of the state's dtype.
// orders: random gate orders tried (0: by state size, -1: none), both for
// splitting each pass into blocks and for re-planning the whole circuit.
constexpr int kMaxPassOrders = 64;
std::vector<PassGroup> plan_passes(const std::vector<Block> &gates, int pass_qubits, int max_fused, int n, int T0,
                                   const int *phys, int orders = 0);
// Every candidate plan_passes compares (the three outer-qubit strategies,
// then the order search on the cheapest of them), in that order.
std::vector<std::vector<PassGroup>> pass_plan_candidates(const std::vector<Block> &gates, int pass_qubits,
                                                         int max_fused, int n, int T0, const int *phys, int orders);
// Model time of a pass plan in HBM round trips of the state (the planner's
// objective).
double pass_plan_cost(const std::vector<PassGroup> &plan);
// A controlled block as a dense unitary on targets + controls (controls
// become the high bits of the index); uncontrolled blocks are returned as is.
Block densify(const Block &b);
// The block a group becomes, without its matrix when it spans two or more
// qubits (targets, controls, width, gate count and diagonality only).
Block group_shape(const std::vector<Block> &gates, const Group &g);
uint64_t qubit_mask(const Block &b);

// Algorithmic HBM bytes / flops of a sweep (physical bit positions).
double block_bytes(int n, int dtype, const Block &b, const int *phys_t, const int *phys_c);
double block_flops(int n, const Block &b);

// Learned cost model (sv_costmodel.hip): feature row of a sweep, the record
// a plan block would produce, and ranking of greedy plans of width 1..max_fused.
void sweep_features(int n, int dtype, const sv_sweep_record &r, float *f);
sv_sweep_record block_record(int n, int dtype, const Block &b, int precision);
// Rank greedy widths 1..max_fused and the learned pass plan (gates: logical,
// phys: the state's map or nullptr); chosen = width, 0 for the pass plan,
// whose plan (on the pre-fused gate list) goes to *pass_plan_out.
int rank_plans(sv_costmodel *m, int n, int dtype, const std::vector<Block> &gates, int max_fused, int precision,
               int &chosen, float *pred_ms, const int *phys, std::vector<PassGroup> *pass_plan_out);
uint64_t costmodel_version(const sv_costmodel *m);
// Learned choice among pass plans (sv_costmodel.hip): candidates of 6, 7 and
// 8 pass qubits over `orders` gate orders on the (pre-fused) gate list, each
// kernel pass given the tile width the model predicts fastest.  phys: the
// state's logical -> physical map (nullptr: identity).  On success `plan`
// holds the winner and *pred_ms its predicted time.
int learned_pass_plan(sv_costmodel *m, int n, int dtype, int precision, const std::vector<Block> &gates,
                      int max_fused, const int *phys, int orders, std::vector<PassGroup> &plan, double *pred_ms);
// The sweep record a kernel pass of a plan would produce (physical tile bits
// from phys), for the tile width T.
sv_sweep_record pass_record(int n, int dtype, int precision, const PassGroup &w, const int *phys, int T);

// ---------------------------------------------------------------------------
// Kernel launchers (device code in the .hip sources).  All pointers are
// device pointers unless named h_*.  Qubit positions are PHYSICAL bits.
// ---------------------------------------------------------------------------
hipError_t launch_reset(void *st, int n, int dtype, hipStream_t s);

// k = 1 dense gate with controls; U by value.
hipError_t launch_gate1(void *st, int n, int dtype, const cd U[4], int t, const int *ctl, int c,
                        hipStream_t s);
// one-target diagonal gate diag(d0, d1) with controls.
hipError_t launch_diag1(void *st, int n, int dtype, cd d0, cd d1, int t, const int *ctl, int c,
                        hipStream_t s);
// dense k-target gate (k <= 6) with controls; d_U = device copy of the matrix
// in the state's precision (complex float or double, row-major).
hipError_t launch_gatek(void *st, int n, int dtype, const void *d_U, int k, const int *tgt,
                        const int *ctl, int c, int precision, hipStream_t s);
// Matrix-core path for k = 4..6 (tile of 2^mfma_tile_log amplitudes, -1 if none).
int mfma_tile_log(int dtype, int k);
hipError_t launch_dense_mfma(void *st, int n, int dtype, const void *d_U, int k, const int *tgt, const int *ctl,
                             int c, hipStream_t s);
// complex64 k = 5, 6 with the three-term BF16 split (needs n - c >= 12).
hipError_t launch_dense_bf16x3(void *st, int n, const void *d_U, int k, const int *tgt, const int *ctl, int c,
                               hipStream_t s);
// Which kernel launch_gatek uses (an sv_sweep_kind).
// Whether a dense 3-target block runs as a 4-target one (U (x) I) because the
// matrix-core path then applies.
bool pads_to_four(int n, int dtype, int c, int precision);
int dense_path(int n, int dtype, int k, int c, int precision);

hipError_t launch_bitswap(void *st, int n, int dtype, int lo, int hi, int w, hipStream_t s);
// dst[j] = amplitude of logical index first + j, j < count.
hipError_t launch_gather_logical(const void *st, void *dst, int n, int dtype, const int *qmap,
                                 uint64_t first, uint64_t count, hipStream_t s);

// Readouts.  Scratch layout is the launcher's business; sizes are checked by
// the caller through the *_scratch_doubles helpers.
uint64_t marginal_scratch_doubles(int n, int m, const int *phys_q);
hipError_t launch_marginal(const void *st, int n, int dtype, const int *phys_q, int m,
                           double *d_scratch, double *d_out, hipStream_t s);
uint64_t expect_scratch_doubles(int n);
// LDS passes (sv_pass.hip): blocks of four tile slots applied in sequence to
// one tile of the pass's qubits + the lowest free bits.
constexpr int kMaxPassQubits = 8;
struct PassSub {
    uint32_t xc[16];      // tile-local index bits of block row r (bit b of r -> slot of block qubit b)
    uint32_t tslot_m[4];  // insert masks 2^slot - 1 of the block's four slots, ascending
    uint64_t u_off;       // byte offset of the 16 x 16 row-major matrix (state precision) from the matrix base
    uint64_t t_off;       // byte offset of the block's phase terms (PassTerm) from the matrix base
    uint32_t nterm;       // number of phase terms (0: the matrix alone)
    uint32_t nvar;        // matrix variants 2^nvar, selected by the tile's index bits vpos[0..nvar)
    uint8_t vpos[8];
    uint32_t pslot;       // with nterm > 0: this block's row of the per-tile angle table (< kMaxTermBlocks)
    uint32_t pad0b;
    uint64_t pad;
};
// Blocks carrying phase terms per pass (rows of the kernel's per-tile angle
// table in LDS); a pass with more runs as ordinary sweeps.
constexpr int kMaxTermBlocks = 16;
// A split-BF16 pass block without phase terms carries its 16 x 16 matrix
// already split: per lane of the MFMA wave, 3 parts x (real, imaginary
// output rows) x 4 packed BF16 pairs (pass_presplit).
constexpr uint64_t kPresplitBytes = 3 * 2 * 64 * 16;
// Write the split A fragments of the 16 x 16 complex matrix U (row-major,
// FP64, rounded to FP32 first) to dst (kPresplitBytes): the same exact
// three-part BF16 split that the pass kernel applies to per-tile matrices.
void pass_presplit(const std::complex<double> *U, void *dst);
static_assert(sizeof(PassSub) == 128, "pass block descriptor layout");
// One monomial of a per-tile phase: where the tile's outer index bits cover
// omask (physical bits), entry (r, c) of the block matrix gains the angle
// 2 pi turn / 2^64 if the block-local column index c (front) or row index r
// (back) covers smask.  Angles in fixed-point turns add exactly and wrap
// modulo 2 pi by themselves.
struct PassTerm {
    uint64_t omask;
    uint32_t smask;
    uint32_t back;
    uint64_t turn;
};
static_assert(sizeof(PassTerm) == 24, "pass phase term layout");
// Smallest pass tile width (log2 amplitudes) and the width used for a pass of
// nsub blocks on an n-qubit state (the smallest or one more).
int pass_tile_log(int dtype);
int pass_tile_log_for(int n, int dtype, int nsub);
// Sorted physical tile bits of a T-bit pass tile (the pass qubits, at most
// T, + the lowest free bits outside phys_avoid); returns T, or -1 if the pass
// does not fit.
int pass_tile_bits(int n, int T, uint64_t phys_qmask, uint64_t phys_avoid, int *tile_bits);
// phases: some block carries phase terms (selects the kernel that reads them);
// split: complex64 blocks as FP32-accurate split BF16 products (T = 12 only).
hipError_t launch_pass(void *st, int n, int dtype, int T, const int *tile_bits, const void *d_subs, int nsub,
                       const void *d_mats, bool phases, bool split, hipStream_t s);

// Device address and size (in doubles) of the fixed scratch array of the
// allocation-free read-out on `device`, which must be the current device.
int noalloc_scratch(int device, double **ptr, uint64_t *doubles);
// Z strings per launch_expect_z call.
int expect_z_batch();
hipError_t launch_expect_z(const void *st, int n, int dtype, const uint64_t *zmasks, int nt,
                           double *d_scratch, double *d_out, hipStream_t s);
hipError_t launch_expect_xy(const void *st, int n, int dtype, uint64_t xmask, uint64_t yzmask,
                            double *d_scratch, double *d_out2, hipStream_t s);
int sample_log_block(int n);
hipError_t launch_block_sums(const void *st, int n, int dtype, double *d_bsums, hipStream_t s);
// Each shot's block and residual target from nb (a power of two) block totals
// and the shots' uniforms, all on the device (one workgroup).
hipError_t launch_sample_prep(const double *d_bsums, uint64_t nb, const double *d_uniforms, int shots,
                              int64_t *d_blocks, double *d_targets, hipStream_t s);
// Per-shot search inside 2^lbs-amplitude blocks (lbs <= 20).
hipError_t launch_sample_search(const void *st, int n, int dtype, const int64_t *d_blocks,
                                const double *d_targets, int shots, int64_t *d_out, int lbs, hipStream_t s);
// Z strings of one fused read-out.
constexpr int kReadoutMaxZ = 32;
// Fused read-out (one read of the state): marginal over phys_q[0..m) (m = 0:
// none), nt <= 32 Z strings, and the totals of 2^readout_log_block blocks.
// Possible where readout_fusable; scratch of readout_scratch_doubles.
bool readout_fusable(int n, int m, const int *phys_q, int dtype);
int readout_log_block(int n, int m, const int *phys_q, int dtype);
uint64_t readout_scratch_doubles(int n, int m, const int *phys_q, int dtype);
hipError_t launch_readout(const void *st, int n, int dtype, const int *phys_q, int m, const uint64_t *zmasks,
                          int nt, double *d_scratch, double *d_marg, double *d_z, double *d_tot, hipStream_t s);

}  // namespace sv
