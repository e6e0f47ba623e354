// Cell binning (counting sort into cell order) and Verlet-list construction
// (Sec. 1.4).  This translation unit is compiled with -ffp-contract=off: the
// wrap and the minimum-image distance are evaluated operation by operation,
// so the neighbour set equals the brute-force definition bit for bit.
#include <math.h>

#include "md_internal.h"

namespace {

// Per-atom kernels run 256-thread blocks, each covering 4 work tiles of 64
// atoms (one wavefront per tile).  Logical blocks are remapped per XCD.
struct AtomSlot {
  int tile;
  int lane;
  bool valid;
};

__device__ __forceinline__ AtomSlot atom_slot(int n_tiles) {
  const int nlb = (n_tiles + 3) / 4;
  const int lb = md_remap_block(nlb);
  AtomSlot s;
  s.tile = lb * 4 + (int)(threadIdx.x / MD_WAVE);
  s.lane = threadIdx.x & (MD_WAVE - 1);
  s.valid = (lb < nlb) && (s.tile < n_tiles);
  return s;
}

__device__ __forceinline__ bool skip_rebuild(int mode, const md_ctl_dev* ctl) {
  return mode == MD_IF_FLAGGED && ctl->rebuild == 0;
}

__device__ __forceinline__ int cell_coord(double x, double lo, double inv_w, int nc) {
  double q = floor((x - lo) * inv_w);
  if (!(q >= 0.0)) return 0;  // also catches NaN
  if (q >= (double)nc) return nc - 1;
  return (int)q;
}

// ---------------------------------------------------------------------------
// 1. wrap, cell index, histogram; the last block scans the histogram.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_count(md_batch b, int mode, double4* pos,
                                                             int* cell_of, int* counts,
                                                             int* cell_start, md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const AtomSlot s = atom_slot(b.n_tiles);
  if (s.valid) {
    const md_tile T = b.tiles[s.tile];
    if (s.lane < T.count) {
      const int i = T.first + s.lane;
      const md_domain& D = b.domains[T.rep];
      double4 p = pos[i];
      double x[3] = {p.x, p.y, p.z};
      int c[3], bad = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!isfinite(x[a])) bad |= MD_FLAG_NONFINITE;
        if (D.periodic[a]) {
          // x <- x - L floor((x - lo) / L); a result of lo + L goes to lo.
          double y = x[a] - D.len[a] * floor((x[a] - D.lo[a]) / D.len[a]);
          if (y >= D.lo[a] + D.len[a]) y = D.lo[a];
          x[a] = y;
        } else if (x[a] < D.lo[a] || x[a] > D.lo[a] + D.len[a]) {
          bad |= MD_FLAG_WALL;
        }
        c[a] = cell_coord(x[a], D.lo[a], D.inv_w[a], D.nc[a]);
      }
      if (bad) md_flag(ctl, bad);
      const int cell = D.cell_off + (c[0] * D.nc[1] + c[1]) * D.nc[2] + c[2];
      pos[i] = make_double4(x[0], x[1], x[2], p.w);
      cell_of[i] = cell;
      atomicAdd(&counts[cell], 1);
    }
  }
  if (md_last_block(&ctl->done[MD_DONE_BIN])) {
    // Exclusive scan of counts into cell_start; counts are reset for the scatter.
    __shared__ int part[MD_ATOM_BLOCK];
    const int nc = b.n_cells, tid = threadIdx.x;
    const int chunk = (nc + MD_ATOM_BLOCK - 1) / MD_ATOM_BLOCK;
    const int beg = tid * chunk, end = min(nc, beg + chunk);
    int sum = 0;
    for (int k = beg; k < end; ++k) sum += counts[k];
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int k = 0; k < MD_ATOM_BLOCK; ++k) {
        int v = part[k];
        part[k] = run;
        run += v;
      }
      cell_start[nc] = run;
      ctl->done[MD_DONE_BIN] = 0u;
      ctl->n_rebuilds += 1;
    }
    __syncthreads();
    int run = part[tid];
    for (int k = beg; k < end; ++k) {
      const int v = counts[k];
      cell_start[k] = run;
      run += v;
      counts[k] = 0;
    }
  }
}

// 2. scatter atom indices into their cell segments (arbitrary order inside a cell).
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_scatter(md_batch b, int mode,
                                                               const int* cell_of, int* counts,
                                                               const int* cell_start, int* src,
                                                               const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const AtomSlot s = atom_slot(b.n_tiles);
  if (!s.valid) return;
  const md_tile T = b.tiles[s.tile];
  if (s.lane >= T.count) return;
  const int i = T.first + s.lane;
  const int c = cell_of[i];
  const int k = atomicAdd(&counts[c], 1);
  src[cell_start[c] + k] = i;
}

// 3. order each cell by atom id (rank sort inside the cell segment) and gather
//    the atom records into the sorted copies.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_gather(
    md_batch b, int mode, const int* cell_of, int* counts, const int* cell_start, const int* src,
    const double4* pos, const double* vel, const int* id, double4* pos_s, double* vel_s,
    int* id_s, const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const AtomSlot s = atom_slot(b.n_tiles);
  if (!s.valid) return;
  const md_tile T = b.tiles[s.tile];
  if (s.lane >= T.count) return;
  const int slot = T.first + s.lane;
  const int n = b.n_atoms;
  const int a = src[slot];
  const int c = cell_of[a];
  const int beg = cell_start[c], end = cell_start[c + 1];
  const int my = id[a];
  int rank = 0;
  for (int k = beg; k < end; ++k) {
    const int o = src[k];
    const int io = id[o];
    rank += (io < my) || (io == my && o < a);
  }
  const int dst = beg + rank;
  pos_s[dst] = pos[a];
  vel_s[dst] = vel[a];
  vel_s[n + dst] = vel[n + a];
  vel_s[2 * n + dst] = vel[2 * n + a];
  id_s[dst] = my;
  if (slot == beg) counts[c] = 0;
}

// 4. copy the sorted records back and take them as the displacement reference.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_copyback(
    md_batch b, int mode, const double4* pos_s, const double* vel_s, const int* id_s,
    double4* pos, double* vel, int* id, double* pos_ref, const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const AtomSlot s = atom_slot(b.n_tiles);
  if (!s.valid) return;
  const md_tile T = b.tiles[s.tile];
  if (s.lane >= T.count) return;
  const int i = T.first + s.lane, n = b.n_atoms;
  const double4 p = pos_s[i];
  pos[i] = p;
  vel[i] = vel_s[i];
  vel[n + i] = vel_s[n + i];
  vel[2 * n + i] = vel_s[2 * n + i];
  id[i] = id_s[i];
  pos_ref[i] = p.x;
  pos_ref[n + i] = p.y;
  pos_ref[2 * n + i] = p.z;
}

// ---------------------------------------------------------------------------
// Verlet list: scan the (de-duplicated) 3x3x3 block of cells around each atom.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int stencil_axis(int c, int nc, int periodic, int* out) {
  int m = 0;
  if (periodic) {
    if (nc >= 3) {
      out[m++] = c == 0 ? nc - 1 : c - 1;
      out[m++] = c;
      out[m++] = c == nc - 1 ? 0 : c + 1;
    } else if (nc == 2) {
      out[m++] = 0;
      out[m++] = 1;
    } else {
      out[m++] = 0;
    }
  } else {
    if (c > 0) out[m++] = c - 1;
    out[m++] = c;
    if (c < nc - 1) out[m++] = c + 1;
  }
  return m;
}

__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_build(md_batch b, int mode, const double4* pos,
                                                         const int* cell_start, int* neigh,
                                                         int* nneigh, int max_neigh, int lanes_log2,
                                                         int npad, double rns2,
                                                         md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const AtomSlot s = atom_slot(b.n_tiles);
  int cnt = 0;
  if (s.valid) {
    const md_tile T = b.tiles[s.tile];
    if (s.lane < T.count) {
      const int i = T.first + s.lane;
      const md_domain& D = b.domains[T.rep];
      const double4 p = pos[i];
      const int cx = cell_coord(p.x, D.lo[0], D.inv_w[0], D.nc[0]);
      const int cy = cell_coord(p.y, D.lo[1], D.inv_w[1], D.nc[1]);
      const int cz = cell_coord(p.z, D.lo[2], D.inv_w[2], D.nc[2]);
      int sx[3], sy[3], sz[3];
      const int mx = stencil_axis(cx, D.nc[0], D.periodic[0], sx);
      const int my = stencil_axis(cy, D.nc[1], D.periodic[1], sy);
      const int mz = stencil_axis(cz, D.nc[2], D.periodic[2], sz);
      const int lanes = 1 << lanes_log2;
      for (int ix = 0; ix < mx; ++ix)
        for (int iy = 0; iy < my; ++iy)
          for (int iz = 0; iz < mz; ++iz) {
            const int cell = D.cell_off + (sx[ix] * D.nc[1] + sy[iy]) * D.nc[2] + sz[iz];
            const int jb = cell_start[cell], je = cell_start[cell + 1];
            for (int j = jb; j < je; ++j) {
              if (j == i) continue;
              const double4 q = pos[j];
              double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
              if (D.periodic[0]) dx = dx - D.len[0] * rint(dx * D.inv_len[0]);
              if (D.periodic[1]) dy = dy - D.len[1] * rint(dy * D.inv_len[1]);
              if (D.periodic[2]) dz = dz - D.len[2] * rint(dz * D.inv_len[2]);
              const double r2 = (dx * dx + dy * dy) + dz * dz;
              if (r2 < rns2) {
                if (cnt < max_neigh)
                  neigh[((size_t)(cnt >> lanes_log2) * npad + i) * lanes + (cnt & (lanes - 1))] = j;
                ++cnt;
              }
            }
          }
      nneigh[i] = cnt < max_neigh ? cnt : max_neigh;
      if (cnt > max_neigh) md_flag(ctl, MD_FLAG_NEIGH_OVERFLOW);
    }
  }
  // One atomic per wavefront for the running maximum of the list length.
  int m = cnt;
#pragma unroll
  for (int o = MD_WAVE / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, MD_WAVE));
  if ((threadIdx.x & (MD_WAVE - 1)) == 0 && m > 0) atomicMax(&ctl->max_nneigh, m);
}

}  // namespace

static bool batch_ok(const md_batch* b) {
  return b && b->n_rep >= 1 && b->n_atoms >= 0 && b->n_tiles >= 0 && b->n_cells >= 1 &&
         b->tile_atoms == MD_TILE && b->domains && (b->tiles || b->n_tiles == 0);
}

extern "C" int md_bin_cells(const md_batch* b, md_rebuild_mode mode, double* pos, double* vel,
                            int* id, double* pos_ref, int* cell_start, void* ws, void* ctl,
                            void* stream) {
  if (!batch_ok(b) || !pos || !vel || !id || !pos_ref || !cell_start || !ws || !ctl)
    return MD_ERR_ARG;
  if (mode != MD_ALWAYS && mode != MD_IF_FLAGGED) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  const md_ws_layout L = md_ws_plan(b);
  char* w = (char*)ws;
  int* cell_of = (int*)(w + L.cell_of);
  int* src = (int*)(w + L.src);
  int* counts = (int*)(w + L.counts);
  double4* pos_s = (double4*)(w + L.pos_s);
  double* vel_s = (double*)(w + L.vel_s);
  int* id_s = (int*)(w + L.id_s);
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(md_grid_blocks((b->n_tiles + 3) / 4)), block(MD_ATOM_BLOCK);
  hipLaunchKernelGGL(k_bin_count, grid, block, 0, st, *b, (int)mode, (double4*)pos, cell_of,
                     counts, cell_start, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_scatter, grid, block, 0, st, *b, (int)mode, cell_of, counts,
                     cell_start, src, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_gather, grid, block, 0, st, *b, (int)mode, cell_of, counts,
                     cell_start, src, (const double4*)pos, vel, id, pos_s, vel_s, id_s, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_copyback, grid, block, 0, st, *b, (int)mode, pos_s, vel_s, id_s,
                     (double4*)pos, vel, id, pos_ref, c);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" int md_build_neighbors(const md_batch* b, md_rebuild_mode mode, const double* pos,
                                  const int* cell_start, const md_nlist* nl, void* ctl,
                                  void* stream) {
  if (!batch_ok(b) || !pos || !cell_start || !nl || !nl->neigh || !nl->nneigh || !ctl)
    return MD_ERR_ARG;
  if (mode != MD_ALWAYS && mode != MD_IF_FLAGGED) return MD_ERR_ARG;
  int lg = -1;
  for (int k = 0; k <= 4; ++k)
    if (nl->lanes == (1 << k)) lg = k;
  if (lg < 0 || nl->max_neigh < nl->lanes || nl->max_neigh % nl->lanes) return MD_ERR_ARG;
  if (!(b->r_ns > 0.0)) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  const dim3 grid(md_grid_blocks((b->n_tiles + 3) / 4)), block(MD_ATOM_BLOCK);
  hipLaunchKernelGGL(k_build, grid, block, 0, (hipStream_t)stream, *b, (int)mode,
                     (const double4*)pos, cell_start, nl->neigh, nl->nneigh, nl->max_neigh, lg,
                     md_npad(b->n_atoms), b->r_ns * b->r_ns, (md_ctl_dev*)ctl);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
