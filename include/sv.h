/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector gate-application library.
 *
 * The library holds one n-qubit state vector of 2^n complex amplitudes in HBM
 * and applies quantum gates to it, then reads it out as probabilities, Pauli
 * expectation values or samples.  The operations follow the paper's statement
 * of state-vector simulation (Sec. 2.1 "State-Vector Simulation" and
 * "Measurement and Sampling"; Sec. 2.2 for the shot-based readout): a state
 * of 2^n amplitudes, unitary gates applied through their tensor product with
 * identities, a one-qubit gate as a 2x2 matrix acting on amplitude pairs,
 * fusion of several gates into one operation, and measurement that draws
 * bitstrings from the distribution the amplitudes define.
 *
 * Conventions (all entry points)
 *  - Qubit q is bit q of the amplitude index (little-endian).  A k-target gate
 *    matrix is 2^k x 2^k, row-major, complex numbers as interleaved (re, im)
 *    doubles; bit b of its row/column index belongs to targets[b].
 *  - Controls act on |1>: the gate is applied to the amplitudes whose control
 *    bits are all 1 and leaves the others unchanged.
 *  - Amplitudes are stored interleaved (re, im): complex64 = 2 x float,
 *    complex128 = 2 x double.  The device buffer is 256-byte aligned.
 *  - Qubit arguments name LOGICAL qubits.  sv_swap_bits() changes the
 *    physical layout and the logical->physical map; every other call
 *    translates through that map, so results never depend on the layout.
 *  - Host buffers are owned by the caller and only touched during the call.
 *    Gate application is stream-ordered and asynchronous; calls that return
 *    host data synchronise the handle's stream before returning.
 *  - Every entry point returns an sv_status.  On failure nothing has been
 *    launched and sv_last_error() gives a message (thread-local).  Argument
 *    checks run on the host before any HIP call, so they work without a GPU.
 *  - A handle must not be used by two threads at once.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sv_status {
    SV_OK = 0,
    SV_EINVAL = -1,       /* bad argument (range, duplicate qubit, null pointer, ...) */
    SV_ENOMEM = -2,       /* device or host allocation failed / state larger than allowed */
    SV_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed */
    SV_EUNSUPPORTED = -4  /* valid request this build does not implement */
} sv_status;

typedef enum sv_dtype {
    SV_C64 = 0,   /* complex64: FP32 re/im, 8 bytes per amplitude */
    SV_C128 = 1   /* complex128: FP64 re/im, 16 bytes per amplitude */
} sv_dtype;

#define SV_MAX_QUBITS 40
#define SV_MAX_TARGETS 6
#define SV_MAX_CONTROLS 8

/* Gate kinds of sv_gate.kind.  Rotations are R_P(t) = exp(-i t P / 2);
 * SV_P(phi) = diag(1, e^{i phi}); SV_U3(t, f, l) =
 * [[cos t/2, -e^{il} sin t/2], [e^{if} sin t/2, e^{i(f+l)} cos t/2]]. */
typedef enum sv_gate_kind {
    SV_GATE_H = 0,
    SV_GATE_X = 1,
    SV_GATE_Y = 2,
    SV_GATE_Z = 3,
    SV_GATE_S = 4,
    SV_GATE_T = 5,
    SV_GATE_RX = 6,
    SV_GATE_RY = 7,
    SV_GATE_RZ = 8,
    SV_GATE_P = 9,
    SV_GATE_U3 = 10,
    SV_GATE_MATRIX = 11  /* dense 2^k x 2^k matrix given by sv_gate.matrix */
} sv_gate_kind;

/* One gate of a circuit.  Named kinds have exactly one target; SV_GATE_MATRIX
 * has 1..SV_MAX_TARGETS.  Any kind may carry up to SV_MAX_CONTROLS controls
 * (CNOT = X with one control, CZ = Z with one control, CP = P with one
 * control).  `matrix` is read during the call only. */
typedef struct sv_gate {
    int32_t kind;
    int32_t num_targets;
    int32_t num_controls;
    int32_t targets[SV_MAX_TARGETS];
    int32_t controls[SV_MAX_CONTROLS];
    double params[3];
    const double *matrix;
} sv_gate;

/* How sv_apply_circuit groups gates into sweeps over the state (paper Sec. 2.1:
 * fusion groups gate applications into one operation, raising the linear
 * algebra size and moving the sweep from bandwidth-bound towards balanced). */
typedef enum sv_plan_mode {
    SV_PLAN_PLAIN = 0,    /* one sweep per gate */
    SV_PLAN_GREEDY = 1,   /* greedy dependency-aware fusion into <= max_fused-qubit blocks */
    SV_PLAN_LEARNED = 2,  /* candidate plans ranked by the attached cost model: greedy widths
                             1..max_fused, and LDS pass plans (as SV_PLAN_PASSES) of 6, 7 and 8
                             pass qubits over several gate orders, each kernel pass with the
                             tile width the model predicts fastest.  The winner is kept on the
                             handle per circuit structure (and model version), so a circuit
                             applied again is not ranked again.  Falls back to SV_PLAN_GREEDY
                             without a usable model */
    SV_PLAN_PASSES = 3    /* greedy dependency-aware grouping into passes of <= pass_qubits
                             qubits; a pass moves the state through LDS once and applies
                             its gates there as a sequence of fused 4-qubit blocks on the
                             matrix cores in the state's own precision (gates on more
                             than 4 qubits, and states below the pass tile, run as greedy
                             <= max_fused-qubit sweeps).  sv_apply_circuit only. */
} sv_plan_mode;

typedef enum sv_precision {
    SV_PREC_NATIVE = 0,   /* complex64: FP32 arithmetic; complex128: FP64 */
    SV_PREC_BF16X3 = 1,   /* complex64 fused blocks of 5-6 qubits: three-term BF16 split
                             products on the matrix cores, FP32 accumulation (relative
                             error ~2^-16 per product); other blocks and complex128
                             run as SV_PREC_NATIVE */
    SV_PREC_BF16X6 = 2    /* complex64 LDS-pass blocks (SV_PLAN_PASSES): every FP32 operand
                             split exactly into three BF16 parts, each real product taken
                             as the six largest of the nine part products on the BF16
                             matrix cores with FP32 accumulation (dropped terms below
                             2^-23 relative per product: FP32-accurate); other sweeps and
                             complex128 run as SV_PREC_NATIVE */
} sv_precision;

typedef struct sv_plan_opts {
    int32_t mode;         /* sv_plan_mode */
    int32_t max_fused;    /* 1..6: widest fused block (greedy / learned; passes' fallback) */
    int32_t precision;    /* sv_precision */
    int32_t pass_qubits;  /* SV_PLAN_PASSES: 4..8 qubits per pass, 0 for 8; else must be 0 */
    int32_t pass_orders;  /* SV_PLAN_PASSES: seeded random gate orders (consistent with the circuit's
                             dependencies) tried when splitting a pass into blocks, beside circuit order and
                             its reverse, and for re-planning the whole circuit; the cheapest result in the
                             pass cost model is kept.  0: by state size (16 from 32 qubits, else none), -1:
                             none, 1..64; else must be 0 */
    int32_t pass_tile;    /* SV_PLAN_PASSES: log2 amplitudes of every kernel pass's LDS tile: 0 = by the
                             pass's blocks; else the smallest tile (12 complex64, 11 complex128) or twice
                             it (complex128, and complex64 with SV_PREC_NATIVE); else must be 0 */
} sv_plan_opts;

/* Counters filled by sv_apply_circuit / sv_apply_plan (may be NULL). */
typedef struct sv_run_stats {
    int64_t gates;              /* gates of the input circuit (unfused count) */
    int64_t sweeps;             /* kernels launched over the state */
    int64_t fused_blocks;       /* sweeps that apply more than one gate */
    double algorithmic_bytes;   /* HBM bytes the sweeps must move (128-byte lines) */
    double flops;               /* real floating-point operations of the sweeps */
} sv_run_stats;

typedef struct sv_state *sv_handle;
typedef struct sv_plan *sv_plan_handle;

/* Thread-local message of the last failed call ("" if none).  Never NULL. */
const char *sv_last_error(void);

/* Bytes of an n-qubit state of dtype: 2^n * 8 (complex64) or 2^n * 16
 * (complex128); the FP32 case is the paper's 2^(n-27) GiB (Sec. 1). */
int sv_state_bytes(int n, int dtype, uint64_t *bytes);

/* Allocate a state of n qubits (1..SV_MAX_QUBITS) on the current HIP device
 * and set it to |0...0>: the complex vector of dimension 2^n of the paper's
 * state-vector representation (Sec. 2.1 "State-Vector Simulation"), 2^(n-27)
 * GiB in complex64 (Sec. 1).  Amplitude 0 is 1, all others 0.  The library
 * owns the memory; sv_destroy frees it.  SV_ENOMEM if the state does not
 * fit in free device memory (or exceeds the SV_MAX_DEVICE_BYTES environment
 * limit, checked on the host first). */
int sv_create(int n, int dtype, sv_handle *out);

/* Wrap caller-owned device memory (e.g. a torch tensor) of `bytes` >=
 * sv_state_bytes(n, dtype), 16-byte aligned, and set it to |0...0>.  The caller
 * keeps the memory alive until sv_destroy.  `stream` is a hipStream_t (NULL =
 * default stream) on which all work of this handle is ordered. */
int sv_create_on(void *device_ptr, uint64_t bytes, int n, int dtype, void *stream, sv_handle *out);

/* Release the handle (and the state if the library allocated it). */
int sv_destroy(sv_handle h);

/* Change the stream work of this handle is ordered on (NULL = default). */
int sv_set_stream(sv_handle h, void *stream);

/* Block until all work queued on the handle's stream has finished. */
int sv_synchronize(sv_handle h);

/* |psi> <- |0...0> and identity qubit map.  One write sweep. */
int sv_reset(sv_handle h);

/* Apply one gate: U is 2^k x 2^k (k = num targets, 1..6) interleaved FP64,
 * `controls` may be NULL when c == 0.  Paper Sec. 2.1: the gate acts through
 * the tensor product of U with identities on the other qubits. */
int sv_apply_gate(sv_handle h, const double *U, const int *targets, int k, const int *controls, int c);

/* Apply a gate list in order, grouped into sweeps as `opts` says (NULL =
 * plain).  All gates are validated before anything is launched. */
int sv_apply_circuit(sv_handle h, const sv_gate *gates, int ngates, const sv_plan_opts *opts,
                     sv_run_stats *stats);

/* Exchange physical index-bit fields [lo, lo+width) and [hi, hi+width)
 * (1 <= width <= 6, lo + width <= hi, hi + width <= n), in place: the
 * single-device part of the global/local qubit exchange a distributed
 * state-vector simulator performs (paper Sec. 2.1, Sec. 2.5).  The logical
 * state is unchanged; the logical->physical map is updated.  Bit-exact. */
int sv_swap_bits(sv_handle h, int lo, int hi, int width);

/* map[q] = physical index bit currently holding logical qubit q (n entries). */
int sv_qubit_map(sv_handle h, int *map);

/* Marginal distribution over logical qubits Q[0..m) (0 <= m <= min(n, 30)):
 * out[x] = sum of |a_i|^2 over i whose qubit Q[b] equals bit b of x; 2^m
 * doubles.  These are the probabilities with which a measurement of the
 * qubits Q returns the bitstring x (Sec. 2.1 "Measurement and Sampling":
 * the amplitudes determine the outcome distribution; the squared moduli of
 * a qubit's amplitudes are its outcome probabilities, Sec. 2.1 "Classical
 * Bits and Qubits").  m = 0 gives the squared norm.  FP64 accumulation for both
 * dtypes.  Synchronises. */
int sv_probabilities(sv_handle h, const int *qubits, int m, double *out);

/* Expectation values <psi|P|psi> of Pauli strings, the quantities shots are
 * repeated to estimate (Sec. 2.1 "Measurement and Sampling") and that the
 * simulator's read-out functions return for each task (Sec. 2.5); here they
 * are computed exactly from the amplitudes.  terms[t] is a string of
 * n characters from "IXYZ" (lower case accepted), character q acting on
 * logical qubit q.  out[t] receives the real part (the imaginary part of a
 * Hermitian expectation is zero up to rounding).  FP64 accumulation.
 * Z-only strings are evaluated together in one read sweep.  Synchronises. */
int sv_expect_pauli(sv_handle h, const char *const *terms, int nterms, double *out);

/* Largest nterms of sv_expect_pauli_noalloc. */
#define SV_NOALLOC_MAX_TERMS 256

/* sv_expect_pauli for callers that cannot allocate memory during the call
 * (serving loops that evaluate expectation values of one state again and
 * again, code that must not call hipMalloc): the same kernels and the same
 * results, but the partial sums live in a fixed device array of the library
 * (1 MiB + 4 KiB on every GPU it runs on, held until the process ends) and
 * the results come back through a host copy straight into `out`: no
 * hipMalloc, hipFree, pinned or heap allocation on the success path.
 * nterms: 0..SV_NOALLOC_MAX_TERMS, SV_EINVAL beyond (and for the argument
 * errors of sv_expect_pauli).  All calls on one GPU share that array, so
 * calls that overlap in time on one GPU (other threads, other handles on
 * the same device) race and must be serialised by the caller; one thread's
 * calls cannot overlap, since each synchronises before returning.  No slot
 * of the array has to start at zero: each call writes every slot it reads. */
int sv_expect_pauli_noalloc(sv_handle h, const char *const *terms, int nterms, double *out);

/* Draw `shots` outcomes (paper Sec. 2.1 "Measurement and Sampling"): for
 * uniform u_s in [0, 1) (caller-drawn), the outcome is the smallest logical
 * basis index x with CDF(x) > u_s * norm, CDF accumulated in FP64 over
 * physical index order (identical to logical order under the identity map).
 * out[s] is the logical bitstring (bit q = qubit q).  Synchronises. */
int sv_sample(sv_handle h, const double *uniforms, int shots, int64_t *out);

/* Draw `shots` outcomes as sv_sample does, with the uniforms taken from the
 * library's own seeded stream: u_s = sv_uniforms(seed, s) for s = 0..shots-1
 * (the paper's benchmarks sample 1000 shots per circuit, Sec. 2.2).  The same
 * seed gives the same outcomes on every call and device.  out: `shots`
 * int64 host values.  Synchronises. */
int sv_sample_seeded(sv_handle h, int shots, uint64_t seed, int64_t *out);

/* The three read-outs of Sec. 2.1 "Measurement and Sampling" of one state in
 * one call: the marginal over qubits[0..m) as sv_probabilities (probs: 2^m
 * doubles; NULL with m = 0 for none), the expectation values of nterms Pauli
 * strings as sv_expect_pauli (expect: nterms doubles; nterms = 0 for none),
 * and `shots` outcomes for the caller's uniforms as sv_sample (samples:
 * shots int64; shots = 0 for none).  Where every string is a Z string (at
 * most 32 of them), the state has at least 14 qubits and the marginal's bits
 * allow it (none of the index bits 9..11 of complex64 or 8..11 of
 * complex128, counted in physical positions), the three share one read of
 * the state: the marginal's partial sums, the strings' partial sums and the
 * totals of 2^12..2^14-amplitude blocks come from one sweep.  Otherwise the
 * three run one after another.  Results equal those of the separate calls
 * up to the order of FP64 additions (shots can differ only where a uniform
 * falls within rounding of a CDF step).
 * Argument errors as in the separate calls.  Synchronises. */
int sv_readout(sv_handle h, const int *qubits, int m, double *probs, const char *const *terms, int nterms,
               double *expect, const double *uniforms, int shots, int64_t *samples);

/* The library's uniform stream, host only (no device work): out[j] = u_{first+j}
 * for j < count, where u_s is the s-th output of SplitMix64 (Steele, Lea, Flood,
 * OOPSLA 2014) started from state `seed`:
 *     z = seed + (s + 1) * 0x9E3779B97F4A7C15 (mod 2^64),
 *     z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9, z = (z ^ (z >> 27)) * 0x94D049BB133111EB,
 *     z = z ^ (z >> 31),  u_s = (z >> 11) * 2^-53  in [0, 1).
 * SV_EINVAL if count < 0 or out is NULL with count > 0. */
int sv_uniforms(uint64_t seed, uint64_t first, int count, double *out);

/* Copy amplitudes [first, first+count) in LOGICAL index order to host memory
 * (count * bytes-per-amplitude bytes, dtype layout): the state vector itself,
 * the result of state-vector simulation (Sec. 2.1 "State-Vector Simulation").
 * `dst` is caller-owned host memory; SV_EINVAL for a range outside [0, 2^n).
 * Synchronises. */
int sv_copy_to_host(sv_handle h, void *dst, uint64_t first, uint64_t count);

/* Overwrite amplitudes [first, first+count) (logical order) from host memory.
 * With a non-identity qubit map only a whole-state copy is allowed; it
 * resets the map to identity.  Synchronises. */
int sv_copy_from_host(sv_handle h, const void *src, uint64_t first, uint64_t count);

/* ---- sweep timing -------------------------------------------------------- */

/* Kernel class of a recorded sweep. */
typedef enum sv_sweep_kind {
    SV_SWEEP_GATE1 = 0,    /* one-target dense gate (controls allowed) */
    SV_SWEEP_DIAG1 = 1,    /* one-target diagonal gate (controls allowed) */
    SV_SWEEP_DENSE = 2,    /* k-target dense block through the LDS tile (VALU) */
    SV_SWEEP_DENSE_MFMA = 3, /* k-target dense block on the matrix cores */
    SV_SWEEP_GROUP = 4,    /* k-target dense block, one group per thread (small n) */
    SV_SWEEP_BITSWAP = 5,  /* index-bit field exchange */
    SV_SWEEP_DENSE_BF16X3 = 6, /* complex64 k-target block, three-term BF16 split on the matrix cores */
    SV_SWEEP_PASS = 7      /* LDS pass: fused 4-qubit blocks on the pass's qubits (k = pass qubits) */
} sv_sweep_kind;

/* One timed sweep (physical bit positions). */
typedef struct sv_sweep_record {
    int32_t kind;            /* sv_sweep_kind */
    int32_t k;               /* targets (bit-field width for SV_SWEEP_BITSWAP) */
    int32_t c;               /* controls */
    int32_t lowest_target;   /* lowest target bit (lo for SV_SWEEP_BITSWAP) */
    int32_t highest_target;  /* highest target bit (hi for SV_SWEEP_BITSWAP) */
    int32_t num_gates;       /* input gates applied by this sweep */
    double bytes;            /* algorithmic HBM bytes */
    double flops;            /* algorithmic: 8 d - 2 per amplitude per dense d x d complex block */
    float ms;                /* HIP-event duration on the handle's stream */
    int32_t precision;       /* sv_precision of the sweep's arithmetic */
    double mfma_flops;       /* real flops a pass executes on the matrix cores (0: other sweeps) */
    int32_t blocks;          /* SV_SWEEP_PASS: fused blocks applied in LDS (0: other sweeps) */
    int32_t term_blocks;     /* SV_SWEEP_PASS: blocks carrying per-tile phase terms */
    int32_t variant_blocks;  /* SV_SWEEP_PASS: blocks staged as per-tile matrix variants */
    int32_t tile_log;        /* SV_SWEEP_PASS: log2 amplitudes of the LDS tile */
    uint64_t tile_mask;      /* SV_SWEEP_PASS: physical index bits of the tile */
} sv_sweep_record;

/* enable != 0: bracket every subsequent sweep of this handle with a pair of
 * HIP events on its stream (the events stay pending until read). */
int sv_profile_enable(sv_handle h, int enable);

/* Synchronise, then move up to `max` recorded sweeps (oldest first) into
 * `out` and their total count into *count; the record buffer is cleared. */
int sv_profile_read(sv_handle h, sv_sweep_record *out, int max, int *count);

/* ---- batches of small circuits in one persistent launch ----------------- */

/* Many independent circuits of uneven width (a parameter sweep) run as one
 * persistent kernel captured in a HIP graph.  Each circuit's state starts at
 * |0...0>; its gates are applied and its Z-string expectation values
 * <psi| Z^{mask} |psi> (FP64 accumulation) are returned.  A circuit that fits
 * one LDS tile runs entirely in LDS; a wider one is cut into passes of LDS
 * tiles ordered through a global work queue (paper Sec. 2.1: the state is 2^n
 * amplitudes and every gate a sweep over them; here the sweeps of a pass are
 * done on-chip). */
typedef struct sv_batch *sv_batch_handle;

/* Tile and fusion choice of a batch (picked by sv_batch_tune or set). */
typedef struct sv_batch_config {
    int32_t tile_bits;   /* log2 amplitudes per LDS tile: complex64 11..13, complex128 11..12 */
    int32_t low_bits;    /* lowest physical bits every tile spans (contiguity), 0..4 */
    int32_t fuse_width;  /* 1: merge runs of one-qubit gates; 2: fuse into <= 2-qubit blocks */
    int32_t reserved;    /* must be 0 */
} sv_batch_config;

/* Create a batch of `ninst` circuits.  Circuit i has nqubits[i] qubits
 * (1..30), gates[i][0..ngates[i]) and nterms[i] (0..64) Z masks zmasks[i][t]
 * (bit q = Z on qubit q).  Supported gates: one target with at most one
 * control, or a two-target SV_GATE_MATRIX without controls.  Later runs must
 * pass gates of the same kinds on the same qubits (parameters may change).
 * `stream` = hipStream_t to run on (NULL: the batch creates its own). */
int sv_batch_create(int dtype, int ninst, const int *nqubits, const sv_gate *const *gates, const int *ngates,
                    const uint64_t *const *zmasks, const int *nterms, void *stream, sv_batch_handle *out);

/* Run the batch: gates = NULL reuses the last parameters, otherwise new
 * gate lists of the created structure.  out receives sum_i nterms[i] values
 * (circuit-major).  Synchronises. */
int sv_batch_run(sv_batch_handle b, const sv_gate *const *gates, double *out);

/* Time every candidate configuration `repeats` times with HIP events and keep
 * the fastest (written to *chosen if not NULL). */
int sv_batch_tune(sv_batch_handle b, int repeats, sv_batch_config *chosen);
int sv_batch_set_config(sv_batch_handle b, const sv_batch_config *cfg);
int sv_batch_get_config(sv_batch_handle b, sv_batch_config *cfg);
/* Milliseconds of the last sv_batch_run's graph launch (HIP events). */
int sv_batch_last_ms(sv_batch_handle b, double *ms);
int sv_batch_destroy(sv_batch_handle b);

/* ---- learned sweep cost model ------------------------------------------ */

/* The best fusion width depends on the machine and the precision (paper Sec.
 * 2.1; Sec. 2.2 quotes different defaults per GPU generation).  A small
 * network learns the run time of one sweep from timings the library records
 * itself (sv_profile_read) and ranks candidate fusion plans by their summed
 * predicted time; SV_PLAN_LEARNED uses it, with the greedy plan as fallback.
 *
 * Network: SV_CM_FEATURES inputs -> SV_CM_HIDDEN ReLU -> SV_CM_HIDDEN ReLU ->
 * 1 output = ln(milliseconds per GB of the sweep's algorithmic HBM traffic);
 * a sweep's predicted time is exp(output) * bytes / 1e9.  Parameters (FP32), in this order:
 * W1 [H x F row-major], b1 [H], W2 [H x H], b2 [H], w3 [H], b3 [1].
 * Training (full-batch Adam on the mean squared error) and gradients run in
 * FP32 on the GPU; prediction runs in FP16 with FP32 accumulation. */
#define SV_CM_FEATURES 16
#define SV_CM_HIDDEN 64

typedef struct sv_costmodel *sv_costmodel_handle;

/* Number of parameters (5313). */
int sv_costmodel_num_params(int *count);
/* New model with He-uniform weights drawn from `seed`, zero biases. */
int sv_costmodel_create(uint64_t seed, sv_costmodel_handle *out);
int sv_costmodel_get_params(sv_costmodel_handle m, float *out);
int sv_costmodel_set_params(sv_costmodel_handle m, const float *in);
/* Loss and gradient at the current parameters over x [n x F], y [n]. */
int sv_costmodel_grad(sv_costmodel_handle m, const float *x, const float *y, int n, float *grad, float *loss);
/* `epochs` full-batch Adam steps (b1 0.9, b2 0.999, eps 1e-8) with rate lr;
 * the Adam moments persist across calls.  *final_loss (may be NULL) is the
 * loss before the last step. */
int sv_costmodel_train(sv_costmodel_handle m, const float *x, const float *y, int n, int epochs, float lr,
                       float *final_loss);
/* FP16 inference: out[i] = network output for feature row i. */
int sv_costmodel_predict(sv_costmodel_handle m, const float *x, int n, float *out);
int sv_costmodel_destroy(sv_costmodel_handle m);

/* Feature rows (count x SV_CM_FEATURES) of recorded sweeps on an n-qubit
 * state of dtype: the sweep's width (targets or pass qubits), controls,
 * gates, lowest and highest target bit, tile bits among the top 8 index
 * bits, dtype, whether it is a pass, its kind, algorithmic bytes, blocks,
 * phase-term and variant blocks, tile width above the smallest, block
 * arithmetic, and the contiguous low tile bits (the length of the runs a
 * pass tile reads), each scaled to about [0, 1]. */
int sv_sweep_features(int n, int dtype, const sv_sweep_record *recs, int count, float *out);

/* Training targets of recorded sweeps: out[i] = ln(ms_i / (bytes_i / 1e9)). */
int sv_sweep_targets(const sv_sweep_record *recs, int count, float *out);

/* Attach a model to a state (NULL detaches); SV_PLAN_LEARNED uses it. */
int sv_set_costmodel(sv_handle h, sv_costmodel_handle m);

/* Rank the candidate plans of a gate list by predicted run time on a fresh
 * n-qubit state of dtype (complex64 passes in SV_PREC_BF16X6 arithmetic):
 * greedy with widest block 1..max_fused, and the best of the LDS pass plans
 * SV_PLAN_LEARNED considers.  predicted_ms (max_fused + 1 entries) receives
 * the prediction for width k at [k-1] and for the pass plan at [max_fused];
 * *chosen is the width with the smallest prediction, 0 for the pass plan, or
 * max_fused if a prediction is not finite. */
int sv_costmodel_rank(sv_costmodel_handle m, int n, int dtype, const sv_gate *gates, int ngates, int max_fused,
                      int *chosen, float *predicted_ms);

/* ---- fusion plans (host only; no GPU needed) ---------------------------- */

/* Build the sweep plan sv_apply_circuit would use for this gate list on an
 * n-qubit state of dtype (logical qubits).  Block matrices are formed in
 * FP64 on the host as the ordered product of the block's gates. */
int sv_plan_create(int n, int dtype, const sv_gate *gates, int ngates, const sv_plan_opts *opts,
                   sv_plan_handle *out);
int sv_plan_num_blocks(sv_plan_handle p, int *nblocks);
/* Block i: k targets and c controls (logical qubits), its 2^k x 2^k FP64
 * matrix (interleaved; may be NULL to skip), and the number of input gates
 * it applies.  targets/controls need room for 6 / 8 entries. */
int sv_plan_block(sv_plan_handle p, int i, int *k, int *targets, int *c, int *controls,
                  double *matrix, int *num_gates);
/* Apply a plan built for this handle's n and dtype. */
int sv_apply_plan(sv_handle h, sv_plan_handle p, sv_run_stats *stats);
int sv_plan_destroy(sv_plan_handle p);

/* Structure of the LDS pass plan (SV_PLAN_PASSES, paper Sec. 2.1 fusion
 * applied as several fused blocks per sweep of the state) that
 * sv_apply_circuit would use for this gate list on a fresh n-qubit state of
 * dtype (every qubit at its own index bit).  Host only: no device work.
 * opts: as for sv_apply_circuit, mode SV_PLAN_PASSES (NULL: defaults).  On
 * success out[0..7] receive: passes; passes run by the pass kernel; blocks in
 * those passes; blocks staged as per-tile matrix variants; blocks carrying
 * per-tile phase terms; ordinary sweeps (passes that fall back to fused
 * sweeps); input gates the plan applies (each input gate exactly once, so
 * this equals ngates); the plan's model time (the planner's objective, in
 * thousandths of one HBM round trip of the state).  SV_EINVAL for invalid
 * gates or options. */
int sv_pass_plan_info(int n, int dtype, const sv_gate *gates, int ngates, const sv_plan_opts *opts, int64_t *out);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
