// Shared host/device layout of a circuit batch (see sv_batch.hip / sv_batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sv {

constexpr int kBatchMaxTileLog = 13;
constexpr int kBatchMaxTerms = 64;
// Threads per workgroup (2^kBatchThreadLog); one workgroup holds one LDS
// tile.  512 threads took 1.5x (complex64) and 1.7x (complex128) longer on
// the 512-circuit HEA batch than 256.
constexpr int kBatchThreadLog = 8;
constexpr int kBatchThreads = 1 << kBatchThreadLog;

struct BInst {
    uint64_t state_off;  // amplitude offset into the batch state buffer (multi-pass circuits)
    int32_t q;
    int32_t npasses;
    int32_t pass0;       // first entry in the pass table
    int32_t nterms;
    int32_t term0;       // first entry in the Z-mask table
    int32_t out0;        // first output slot
    int32_t part0;       // first partial-sum slot (multi-tile last pass)
    int32_t pad;
};

struct BPass {
    uint64_t dep[kBatchMaxTileLog];  // 2^(physical bit) of tile bit b
    uint64_t ins[kBatchMaxTileLog];  // insert masks (ascending tile bits): tile index -> base
    int32_t lp;                      // tile bits of this pass
    int32_t step0;
    int32_t nsteps;
    uint32_t ntiles;
    uint32_t need;                   // finished tiles of earlier passes required before start
    int32_t last;                    // last pass: reduce expectation values instead of storing
    uint32_t mat0;                   // first matrix element of the pass's steps
    uint32_t nmat;                   // matrix elements of the pass's steps, contiguous from mat0
};

// Per-pass copies in LDS, taken at the start of every task: the first
// kBatchStepCache steps, and every matrix when they fit in
// kBatchMatCacheBytes (else the steps read them from global memory).
constexpr int kBatchStepCache = 128;
constexpr int kBatchMatCacheBytes = 8192;

// One in-LDS gate step.  type 0: dense one-qubit on tile bit a; 1: one-qubit
// on tile bit a controlled by tile bit b; 2: dense two-qubit, matrix index bit
// 0 on tile bit a and bit 1 on tile bit b.
struct BStep {
    uint32_t mat;  // offset of the matrix in complex elements
    uint8_t type;
    uint8_t a;
    uint8_t b;
    uint8_t pad;
};

// Dynamic LDS bytes of a batch launch with tiles of 2^tile_log amplitudes of
// amp_bytes each: tile | per-wave partial sums | matrix copy | step copy.
constexpr size_t batch_lds_bytes(int tile_log, size_t amp_bytes)
{
    return (amp_bytes << tile_log) + size_t(kBatchThreads / 64) * 16 * sizeof(double) + kBatchMatCacheBytes +
           kBatchStepCache * sizeof(BStep);
}

struct BTask {
    uint32_t inst;
    uint32_t pass;  // pass index within the circuit
    uint32_t tile;
    uint32_t pad;
};

struct BatchArgs {
    void *states;
    const BInst *inst;
    const BPass *pass;
    const BStep *steps;
    const void *mats;
    const BTask *tasks;
    const uint64_t *zmasks;
    double *partials;
    double *out;
    uint32_t *ctr;  // [0] queue head, [1] error, [2, 2+ninst) tiles done, then finish counts
    uint32_t ntasks;
    uint32_t ninst;
    uint32_t spin_limit;
    int32_t tile_log_max;
};

hipError_t launch_batch(int dtype, const BatchArgs &a, uint32_t grid, size_t lds, hipStream_t s);
hipError_t launch_batch_fill(uint32_t *ctr, uint32_t n, hipStream_t s);
// Persistent grid for the batch kernel with `lds` dynamic bytes per workgroup.
uint32_t batch_grid(int dtype, size_t lds);

}  // namespace sv
