// Internal definitions shared by the HIP translation units of libmd950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md.h"

#define MD_WAVE 64
#define MD_TILE 64           // atoms per work tile (one wavefront at one lane per atom)
#define MD_ATOM_BLOCK 256    // threads per block of the per-atom kernels (4 tiles)
#define MD_XCD 8             // accelerator complex dies on MI355X
#define MD_MAX_LANES 16

// 1 eV / (u angstrom) in angstrom / ps^2.
#define MD_ACCEL 9648.5332157

// Device control block (md_ctl_bytes()).
struct md_ctl_dev {
  unsigned long long dmax_bits;  // max |x - x_ref|^2 of the running drift, as raw bits
  int rebuild;                   // 1: the MD_IF_FLAGGED rebuild kernels do their work
  int step;                      // completed kick-drift steps
  int flags;                     // sticky MD_FLAG_* bits
  int n_rebuilds;
  int max_nneigh;
  int pad;
  unsigned int done[8];          // arrival counters of the last-block reductions
};
enum { MD_DONE_BIN = 0, MD_DONE_VERLET = 1, MD_DONE_FORCE = 2, MD_DONE_ADJ = 3 };

// Offsets of the workspace regions (bytes, 256-aligned).
struct md_ws_layout {
  size_t cell_of, src, counts, pos_s, vel_s, id_s, partial, total;
};

static inline size_t md_align256(size_t x) { return (x + 255) & ~(size_t)255; }

static inline md_ws_layout md_ws_plan(const md_batch* b) {
  md_ws_layout L;
  size_t n = (size_t)b->n_atoms, o = 0;
  L.cell_of = o; o = md_align256(o + 4 * n);
  L.src = o;     o = md_align256(o + 4 * n);
  L.counts = o;  o = md_align256(o + 4 * (size_t)(b->n_cells + 1));
  L.pos_s = o;   o = md_align256(o + 32 * n);
  L.vel_s = o;   o = md_align256(o + 24 * n);
  L.id_s = o;    o = md_align256(o + 4 * n);
  L.partial = o; o = md_align256(o + 8 * MD_EV_LEN * (size_t)b->n_tiles);
  L.total = o;
  return L;
}

static inline int md_npad(int n) { return (n + 63) & ~63; }

// Grid size for `nblocks` logical blocks, rounded up so that the XCD remap below
// is a bijection.
static inline int md_grid_blocks(int nblocks) { return ((nblocks + MD_XCD - 1) / MD_XCD) * MD_XCD; }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Give each XCD a contiguous range of logical blocks, so that spatially adjacent
// tiles (cell order) share an L2.  Returns a value >= nblocks for padding blocks.
__device__ __forceinline__ int md_remap_block(int nblocks) {
  const int per = (nblocks + MD_XCD - 1) / MD_XCD;
  const int b = blockIdx.x;
  return (b % MD_XCD) * per + b / MD_XCD;
}

__device__ __forceinline__ void md_flag(md_ctl_dev* ctl, int bits) { atomicOr(&ctl->flags, bits); }

// Butterfly sum over the whole wavefront; every lane ends with the same value
// (each stage adds a commutative pair, so all lanes round identically).
template <typename T>
__device__ __forceinline__ T md_wave_sum(T v) {
#pragma unroll
  for (int o = MD_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, MD_WAVE);
  return v;
}

// Butterfly sum over aligned groups of G lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T md_group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, MD_WAVE);
  return v;
}

// Deterministic block sum of NV doubles: wave butterflies, then wave 0 adds the
// per-wave results in wave order.  Result valid in thread 0.  `sh` must hold
// NV * (blockDim / 64) doubles.
template <int NV>
__device__ __forceinline__ void md_block_sum(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & (MD_WAVE - 1), wid = threadIdx.x / MD_WAVE;
  const int nw = blockDim.x / MD_WAVE;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = md_wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wid * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = sh[k];
      for (int w = 1; w < nw; ++w) s += sh[w * NV + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Last-block detection: every block calls this once after its global writes.
// Returns true in exactly one block, the last to arrive, after which every
// write of every block is visible to it.  Never waits on other blocks.
__device__ __forceinline__ bool md_last_block(unsigned int* counter) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int prev = atomicAdd(counter, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

// Host-side launch helpers (defined in md_api.cpp).
int md_hip_status(hipError_t e);
#define MD_LAUNCH_CHECK() \
  do {                                                    \
    hipError_t _e = hipGetLastError();                    \
    if (_e != hipSuccess) return md_hip_status(_e);       \
  } while (0)
