// d2q9_launch.hpp -- host-side launchers of the D2Q9 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "d2q9_core.hpp"

namespace lbmp {

// One time step: pull from `fin`, collide, store into `fout` (both the
// post-collision layout).  Sets flag[0] on an unstable site.  The pseudopotential
// form is k.psi_form (also for the moments and diagnostics passes).
hipError_t launch_step(int store, bool walls, const void* fin, void* fout, const StepConst& k,
                       int* flag, hipStream_t s);

// Whether launch_step runs the two-columns-per-lane kernel for this store type
// and lattice width (destination-scaled FP16, even nx).
bool pair_step(int store, int nx);

// Resident workgroups per compute unit of the two-columns-per-lane step (0 if the query fails).
int pair_blocks_per_cu(bool walls);

// Persistent batched step: workgroup i advances lattice inst[i] by `steps`
// steps starting from buffer `parity`; clocks[2i], clocks[2i+1] receive the
// wall clock at the workgroup's start and end.  Stores: F32, F16 local, F16
// destination-scaled; `psi` (kPsiCS / kPsiSS) is shared by all lattices.
hipError_t launch_batch(int store, bool walls, int psi, const BatchInstance* inst, int n, int steps,
                        int parity, unsigned long long* clocks, hipStream_t s);

// Flat batched step: one step of every lattice of a list in one launch over the
// global tile list (tile_start: n+1 prefix sums; wg_first: lattice of each
// workgroup's first tile, indexed by the renumbered workgroup id).  pair: the
// lattices are destination-scaled FP16 with an even nx and are stepped two
// columns per lane (descriptors with 124-column tiles); otherwise one column
// per lane (62-column tiles).
hipError_t launch_batch_flat(int store, bool walls, int psi, bool pair, const BatchInstance* inst,
                             const int* tile_start, const int* wg_first, int ntotal, int parity, hipStream_t s);

// Wavefronts (tiles) per workgroup of launch_batch_flat.
int batch_waves_per_block(int store, bool pair);

// Resident step workgroups per compute unit (0 if the query fails).
int step_blocks_per_cu(int store, bool walls);

// rho and v of the state in `fin` into unpadded [ny][nx] FP32 buffers (NULL allowed).
hipError_t launch_moments(int store, bool walls, const void* fin, const StepConst& k, int* flag,
                          float* rho, float* ux, float* uy, hipStream_t s);

// FP64 reductions of the state in `fin`: per-wave partials, then a fixed-order
// single-block pass into out[kDiagFields].
hipError_t launch_diag(int store, bool walls, const void* fin, const StepConst& k, int* flag,
                       const DiagConst& dg, double* partial, double* out, hipStream_t s);

// Equilibrium initial state into `fout`; flag[0] = kFlagBadInput on invalid input.
hipError_t launch_init(int store, bool walls, const float* rho0, const float* ux0,
                       const float* uy0, void* fout, const StepConst& k, const InitConst& ic, int* flag,
                       hipStream_t s);

// Streaming copy of n16 16-byte elements (attainable-bandwidth reference).
hipError_t launch_copy_probe(const void* src, void* dst, long long n16, hipStream_t s);

}  // namespace lbmp
