// Internal definitions shared by the HIP translation units of libmd950.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md.h"

#define MD_WAVE 64
#define MD_TILE MD_TILE_ATOMS  // atoms per work tile (one wavefront at one lane per atom)
#define MD_ATOM_BLOCK 256    // threads per block of the per-atom kernels (4 tiles)
#define MD_XCD 8             // accelerator complex dies on MI355X
#define MD_MAX_LANES 16

// 1 eV / (u angstrom) in angstrom / ps^2.
#define MD_ACCEL 9648.5332157

// Device control block (md_ctl_bytes()).
#define MD_MAX_ATOM_BLOCKS 4096  // grid cap of the per-atom kernels (grid-stride beyond)
#define MD_DMAX_SLOTS MD_DRIFT_MAX_BLOCKS  // per-block displacement maxima a drifting kernel may publish

struct md_ctl_dev {
  int rebuild;     // 1: the MD_IF_FLAGGED rebuild kernels do their work
  int step;        // current step (advanced by the force pass that follows a kick-drift)
  int flags;       // sticky MD_FLAG_* bits
  int n_rebuilds;
  int max_nneigh;
  int n_dmax;      // valid entries in dmax[] (0 right after a rebuild)
  int step_next;   // step + 1, published by the kick-drift
  int rec_stale;   // 1: positions changed since the last force pass other than by its fused
                   // kick-drift (md_ctl_init, md_bin_cells, md_verlet_step's drift), so FP32
                   // neighbour records carried over in md_drift.rec_in must be remade
  double thr2;     // (half skin)^2 of the last kick-drift; < 0: no criterion
  double pad2;
  double dmax[MD_DMAX_SLOTS];  // per-block max |x - x_ref|^2 of the last drift
};

// Largest per-block displacement of the last drift above the threshold?  Read
// by every block that needs it (each block reduces the <= 4096 maxima itself).
__device__ __forceinline__ bool md_displacement_exceeded(const md_ctl_dev* ctl) {
  const double thr2 = ctl->thr2;
  const int n = ctl->n_dmax;
  int over = 0;
  if (thr2 >= 0.0)
    for (int k = threadIdx.x; k < n; k += blockDim.x) over |= ctl->dmax[k] > thr2;
  return __syncthreads_or(over) != 0;
}

__device__ __forceinline__ void md_flag(md_ctl_dev* ctl, int bits);

// Block 0 of the first force kernel of a step: advance the step counter to the
// value the kick-drift published, and verify the neighbour list: if an atom has
// moved more than half the skin since the list was built and no rebuild followed,
// the list may miss pairs (MD_FLAG_STALE_LIST).
// verify_rec: the call was told its carried FP32 neighbour records are current (no records
// kernel ran); a stale flag then marks the step void (MD_FLAG_STALE_RECORDS).
__device__ __forceinline__ void md_step_bookkeeping(md_ctl_dev* ctl, bool verify_rec = false) {
  if (blockIdx.x != 0) return;
  const bool stale = md_displacement_exceeded(ctl);
  if (threadIdx.x == 0) {
    if (stale) md_flag(ctl, MD_FLAG_STALE_LIST);
    if (verify_rec && ctl->rec_stale) md_flag(ctl, MD_FLAG_STALE_RECORDS);
    ctl->step = ctl->step_next;
    ctl->rec_stale = 0;  // this pass's records are made (the records kernel ran before it)
  }
}

// Offsets of the workspace regions (bytes, 256-aligned).
struct md_ws_layout {
  size_t cell_of, rank, src, sid, counts, scan, pos_s, vel_s, id_s, partial, rec, total;
};

// Blocks of the cell-histogram scan (one segment of cells each).
#define MD_SCAN_BLOCKS 1024

static inline size_t md_align256(size_t x) { return (x + 255) & ~(size_t)255; }

// A well-formed batch descriptor (host check of every entry point).  A batch may hold
// no atoms; its tile array may then be NULL.
static inline bool md_batch_ok(const md_batch* b) {
  return b && b->n_rep >= 1 && b->n_atoms >= 0 && b->n_atoms <= MD_MAX_ATOMS &&
         b->n_tiles >= 0 && b->n_cells >= 1 && b->tile_atoms == MD_TILE && b->domains &&
         (b->tiles || b->n_tiles == 0);
}

static inline md_ws_layout md_ws_plan(const md_batch* b) {
  md_ws_layout L;
  size_t n = (size_t)b->n_atoms, o = 0;
  L.cell_of = o; o = md_align256(o + 4 * n);
  L.rank = o;    o = md_align256(o + 4 * n);
  L.src = o;     o = md_align256(o + 4 * n);
  L.sid = o;     o = md_align256(o + 4 * n);
  L.counts = o;  o = md_align256(o + 4 * (size_t)(b->n_cells + 1));
  L.scan = o;    o = md_align256(o + 4 * (size_t)MD_SCAN_BLOCKS);
  L.pos_s = o;   o = md_align256(o + 32 * n);
  L.vel_s = o;   o = md_align256(o + 24 * n);
  L.id_s = o;    o = md_align256(o + 4 * n);
  L.partial = o; o = md_align256(o + 8 * MD_EV_LEN * (size_t)b->n_tiles);
  L.rec = o;     o = md_align256(o + 16 * n);  // FP32 EAM: fixed-point neighbour records
  L.total = o;
  return L;
}

// nneigh[i] = list length | MD_NN_IMG when the atom's cell stencil crosses a
// periodic boundary (only then do the force passes apply the minimum image).
#define MD_NN_IMG (1 << 30)
#define MD_NN_MASK (MD_NN_IMG - 1)

static inline int md_npad(int n) { return (n + 63) & ~63; }

// Grid size for `nblocks` logical blocks, rounded up so that the XCD remap below
// is a bijection.
static inline int md_grid_blocks(int nblocks) { return ((nblocks + MD_XCD - 1) / MD_XCD) * MD_XCD; }

// Per-atom kernels: 256-thread blocks of 4 tiles, at most MD_MAX_ATOM_BLOCKS blocks
// (a block then strides over logical blocks).
static inline int md_atom_grid(int n_tiles) {
  const int g = md_grid_blocks((n_tiles + 3) / 4);
  return g < MD_MAX_ATOM_BLOCKS ? g : MD_MAX_ATOM_BLOCKS;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Give each XCD a contiguous range of logical blocks, so that spatially adjacent
// tiles (cell order) share an L2.  Returns a value >= nblocks for padding blocks.
__device__ __forceinline__ int md_remap_block(int nblocks) {
  const int per = (nblocks + MD_XCD - 1) / MD_XCD;
  const int b = blockIdx.x;
  return (b % MD_XCD) * per + b / MD_XCD;
}

// Same remap for a grid of gridDim.x blocks striding over nblocks logical blocks:
// the k-th logical block of block b.
__device__ __forceinline__ int md_remap_stride(int nblocks, int k) {
  const int g = gridDim.x;
  const int per = (g + MD_XCD - 1) / MD_XCD;
  const int b = blockIdx.x;
  return ((b % MD_XCD) * per + b / MD_XCD) + k * g;
}

__device__ __forceinline__ void md_flag(md_ctl_dev* ctl, int bits) { atomicOr(&ctl->flags, bits); }

// Walls of md_walls in kernel-argument form (enabled = 0: none).
struct md_walls_dev {
  int enabled, axis;
  double z0, v, top;
};

static inline int md_walls_load(const md_walls* walls, md_walls_dev* w) {
  *w = md_walls_dev{0, 2, 0.0, 0.0, 0.0};
  if (walls && walls->enabled) {
    if (walls->axis < 0 || walls->axis > 2) return MD_ERR_ARG;
    *w = md_walls_dev{1, walls->axis, walls->piston_z0, walls->piston_v, walls->top};
  }
  return MD_OK;
}

// Langevin thermostat in device form: per region the slab bounds, the decay
// c1 = exp(-gamma dt), the noise amplitude c2 = sqrt((1 - c1^2) k_B T / m) in
// angstrom/ps and the mean velocity.
struct md_langevin_dev {
  const int* id;
  unsigned key0, key1;
  int axis, n;
  double lo[MD_MAX_THERMO_REGIONS], hi[MD_MAX_THERMO_REGIONS];
  double c1[MD_MAX_THERMO_REGIONS], c2[MD_MAX_THERMO_REGIONS];
  double u[MD_MAX_THERMO_REGIONS][3];
};

// Host form of md_langevin for one time step and mass (md_verlet.hip); a NULL md_langevin
// gives n = 0 (no thermostat).  MD_ERR_ARG for a malformed one.
int md_langevin_load(const md_langevin* lg, double dt, double inv_mass, md_langevin_dev* L);

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 -> 64-bit
// multiplies with the Weyl key schedule.
__device__ __forceinline__ void md_philox4x32_10(unsigned (&c)[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned a = c[0], b = c[2];
    const unsigned hi0 = __umulhi(0xD2511F53u, a), lo0 = 0xD2511F53u * a;
    const unsigned hi1 = __umulhi(0xCD9E8D57u, b), lo1 = 0xCD9E8D57u * b;
    c[0] = hi1 ^ c[1] ^ k0;
    c[1] = lo1;
    c[2] = hi0 ^ c[3] ^ k1;
    c[3] = lo0;
  }
}

// Three standard normals for (id, step): Box-Muller on the four Philox words.
__device__ __forceinline__ void md_langevin_normals(int id, int step, unsigned k0, unsigned k1,
                                                    double (&z)[3]) {
  unsigned c[4] = {(unsigned)id, (unsigned)step, 0u, 0u};
  md_philox4x32_10(c, k0, k1);
  const double s32 = 2.3283064365386963e-10;  // 2^-32
  const double two_pi = 6.283185307179586;
  const double u0 = ((double)c[0] + 1.0) * s32, u1 = (double)c[1] * s32;
  const double u2 = ((double)c[2] + 1.0) * s32, u3 = (double)c[3] * s32;
  const double r0 = sqrt(-2.0 * log(u0)), r2 = sqrt(-2.0 * log(u2));
  z[0] = __dmul_rn(r0, cos(two_pi * u1));
  z[1] = __dmul_rn(r0, sin(two_pi * u1));
  z[2] = __dmul_rn(r2, cos(two_pi * u3));
}

// The Langevin velocity update of one atom at position x (start of the step); the
// region coordinate is folded into the box on a periodic axis, as the wrap of the
// binning pass does (x - L floor((x - lo) / L), lo + L going to lo).  Products are
// rounded on their own (__dmul_rn: no fused multiply-add), so the separate kick-drift
// kernel and the force pass that fuses it give the same bits whatever each
// compilation contracts.
__device__ __forceinline__ void md_langevin_atom(const md_langevin_dev& L, const md_domain& D,
                                                 int i, int step, const double (&x)[3],
                                                 double (&v)[3]) {
  const int a = L.axis;
  double xa = a == 0 ? x[0] : (a == 1 ? x[1] : x[2]);
  if (D.periodic[a]) {
    xa = xa - __dmul_rn(D.len[a], floor((xa - D.lo[a]) / D.len[a]));
    if (xa >= D.lo[a] + D.len[a]) xa = D.lo[a];
  }
  int r = -1;
  for (int q = L.n - 1; q >= 0; --q)
    if (xa >= L.lo[q] && xa < L.hi[q]) r = q;
  if (r < 0) return;
  double z[3];
  md_langevin_normals(L.id[i], step, L.key0, L.key1, z);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    v[k] = (L.u[r][k] + __dmul_rn(L.c1[r], v[k] - L.u[r][k])) + __dmul_rn(L.c2[r], z[k]);
}

// The integrator's multiply-adds, written as explicit fused operations: the kick
// v + c F, the drift x + dt v and squared norms are then rounded the same way in every
// kernel that computes them (the separate kick-drift and the force passes that fuse it),
// whatever each compilation would contract.
__device__ __forceinline__ double md_kick(double v, double c, double f) { return fma(c, f, v); }
__device__ __forceinline__ double md_norm2(double x, double y, double z) {
  return fma(z, z, fma(y, y, x * x));
}

// The drift of velocity Verlet for one atom: x <- x + dt v (x holds the old
// position on entry), then the walls at t_new: a piston plane z0 + v_p t that
// reflects specularly in its own frame, and a static top wall (Sec. 1.5).  Shared
// by the kick-drift kernel and the force pass that fuses the next kick-drift, so
// both give the same bits.
__device__ __forceinline__ void md_drift_atom(double (&x)[3], double (&v)[3], double dt,
                                              const md_walls_dev& w, double t_new) {
  x[0] = fma(dt, v[0], x[0]);
  x[1] = fma(dt, v[1], x[1]);
  x[2] = fma(dt, v[2], x[2]);
  if (w.enabled) {
    const int a = w.axis;
    const double zp = fma(w.v, t_new, w.z0);
    if (x[a] < zp) {
      x[a] = 2.0 * zp - x[a];
      v[a] = 2.0 * w.v - v[a];
    }
    if (x[a] > w.top) {
      x[a] = 2.0 * w.top - x[a];
      v[a] = -v[a];
    }
  }
}

// |x - x_ref|^2 for the half-skin criterion; NaN counts as infinite (a rebuild,
// and the non-finite flag is raised by the caller).
__device__ __forceinline__ double md_disp2(const double (&x)[3], const double* pos_ref, int i,
                                           int n) {
  const double dx = x[0] - pos_ref[i], dy = x[1] - pos_ref[n + i], dz = x[2] - pos_ref[2 * n + i];
  const double d2 = md_norm2(dx, dy, dz);
  return d2 >= 0.0 ? d2 : INFINITY;
}

// Publish a block's displacement maximum (all threads call; blockDim <= 1024).
// Block 0 also sets the fields the next step's rebuild and force kernels read.
__device__ __forceinline__ void md_publish_dmax(double d2max, int bad, double thr2,
                                                md_ctl_dev* ctl) {
  __shared__ double s_dmax[16];
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d2max = fmax(d2max, __shfl_xor(d2max, o, 64));
  if (__any(bad)) {
    int all = bad;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) all |= __shfl_xor(all, o, 64);
    if (lane == 0) md_flag(ctl, all);
  }
  if (lane == 0) s_dmax[threadIdx.x / 64] = d2max;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = s_dmax[0];
    for (int k = 1; k < (int)(blockDim.x / 64); ++k) m = fmax(m, s_dmax[k]);
    ctl->dmax[blockIdx.x] = m;
    if (blockIdx.x == 0) {  // fields no block of the publishing kernel reads
      ctl->n_dmax = gridDim.x;
      ctl->thr2 = thr2;
      ctl->step_next = ctl->step + 1;
    }
  }
}

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

// Deterministic block sum of NV doubles: wave butterflies, then wave 0 combines
// the per-wave results with a second butterfly (fixed order).  Result valid in
// thread 0.  `sh` must hold NV * (blockDim / 64) doubles; blockDim <= 4096.
template <int NV>
__device__ __forceinline__ void md_block_sum(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & (MD_WAVE - 1), wid = threadIdx.x / MD_WAVE;
  const int nw = blockDim.x / MD_WAVE;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = md_wave_sum(v[k]);
  if (nw == 1) return;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wid * NV + k] = v[k];
  }
  __syncthreads();
  if (wid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = md_wave_sum(lane < nw ? sh[lane * NV + k] : 0.0);
  }
  __syncthreads();
}

// Per-group sums for blocks that process G groups of W wavefronts each (one work
// tile per group): wave butterflies, then thread g*NV + k adds the W wave results
// of group g in wave order.  Returns true in the threads holding out[g*NV + k] in
// `res`.  `sh` must hold NV * (blockDim / 64) doubles.
template <int NV>
__device__ __forceinline__ bool md_group_waves_sum(double (&v)[NV], int waves_per_group,
                                                   double* sh, double& res, int& g, int& k) {
  const int lane = threadIdx.x & (MD_WAVE - 1), wid = threadIdx.x / MD_WAVE;
  const int nw = blockDim.x / MD_WAVE;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = md_wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wid * NV + q] = v[q];
  }
  __syncthreads();
  const int ng = nw / waves_per_group;
  const int tid = threadIdx.x;
  bool have = tid < ng * NV;
  if (have) {
    g = tid / NV;
    k = tid % NV;
    double s = sh[(g * waves_per_group) * NV + k];
    for (int w = 1; w < waves_per_group; ++w) s += sh[(g * waves_per_group + w) * NV + k];
    res = s;
  }
  __syncthreads();
  return have;
}

// Cross-block results are never combined inside a kernel: on MI355X each of the
// 8 XCDs has a private L2, so a device-scope release fence writes dirty L2 lines
// back to memory.  Blocks write partials; a later kernel (stream order makes them
// visible) reduces them.

// Host-side launch helpers (defined in md_api.hip).
int md_hip_status(hipError_t e);

// Kernel timer (md_timer_arm): true once for the armed kernel id, with its events.
bool md_timer_take(int kernel, hipEvent_t* start, hipEvent_t* stop);

// Launch a kernel, bracketed by the timer's events when that kernel id is armed.
#define MD_LAUNCH_TIMED(KID, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                     \
  do {                                                                                  \
    hipEvent_t _t0, _t1;                                                                \
    if (md_timer_take((KID), &_t0, &_t1))                                               \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, _t0, _t1, 0, __VA_ARGS__); \
    else                                                                                \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);              \
  } while (0)
#define MD_LAUNCH_CHECK() \
  do {                                                    \
    hipError_t _e = hipGetLastError();                    \
    if (_e != hipSuccess) return md_hip_status(_e);       \
  } while (0)
