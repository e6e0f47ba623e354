// Cell binning (counting sort into cell order) and Verlet-list construction
// (Sec. 1.4).  This translation unit is compiled with -ffp-contract=off: the
// wrap and the minimum-image distance are evaluated operation by operation,
// so the neighbour set equals the brute-force definition bit for bit.
#include <math.h>

#include "md_internal.h"

namespace {

// Per-atom kernels run 256-thread blocks, each covering 4 work tiles of 64
// atoms (one wavefront per tile).  Logical blocks are remapped per XCD; a block
// strides over logical blocks when the grid is capped.  FOR_ATOMS(i, T) runs
// its body for every atom i of the block's tiles (T the tile).
#define FOR_ATOMS(b, I, T, ...)                                               \
  do {                                                                        \
    const int _nlb = ((b).n_tiles + 3) / 4;                                   \
    const int _lane = threadIdx.x & (MD_WAVE - 1);                            \
    for (int _k = 0;; ++_k) {                                                 \
      const int _lb = md_remap_stride(_nlb, _k);                              \
      if (_lb >= _nlb) break;                                                 \
      const int _t = _lb * 4 + (int)(threadIdx.x / MD_WAVE);                  \
      if (_t >= (b).n_tiles) continue;                                        \
      const md_tile T = (b).tiles[_t];                                        \
      if (_lane >= T.count) continue;                                         \
      const int I = T.first + _lane;                                          \
      __VA_ARGS__                                                             \
    }                                                                         \
  } while (0)

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
// 1. wrap, cell index, histogram.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_count(md_batch b, int mode, double4* pos,
                                                             int* cell_of, int* counts,
                                                             md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  int bad = 0;
  FOR_ATOMS(b, i, T, {
    const md_domain& D = b.domains[T.rep];
    double4 p = pos[i];
    double x[3] = {p.x, p.y, p.z};
    int c[3];
_Pragma("unroll")
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
    const int cell = D.cell_off + (c[0] * D.nc[1] + c[1]) * D.nc[2] + c[2];
    pos[i] = make_double4(x[0], x[1], x[2], p.w);
    cell_of[i] = cell;
    atomicAdd(&counts[cell], 1);
  });
  if (bad) md_flag(ctl, bad);
}

// 2. one block: exclusive scan of the histogram into cell_start; counts reset.
__global__ __launch_bounds__(1024) void k_bin_scan(int n_cells, int mode, int* counts,
                                                    int* cell_start, md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  __shared__ int part[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int chunk = (n_cells + nt - 1) / nt;
  const int beg = min(n_cells, tid * chunk), end = min(n_cells, beg + chunk);
  int sum = 0;
  for (int k = beg; k < end; ++k) sum += counts[k];
  part[tid] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the chunk sums
  for (int o = 1; o < nt; o <<= 1) {
    const int v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - sum;
  for (int k = beg; k < end; ++k) {
    const int v = counts[k];
    cell_start[k] = run;
    run += v;
    counts[k] = 0;
  }
  if (tid == nt - 1) {
    cell_start[n_cells] = part[nt - 1];
    ctl->n_rebuilds += 1;
  }
}

// 3. scatter atom indices into their cell segments (arbitrary order inside a cell).
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_scatter(md_batch b, int mode,
                                                               const int* cell_of, int* counts,
                                                               const int* cell_start, int* src,
                                                               const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  FOR_ATOMS(b, i, T, {
    const int c = cell_of[i];
    const int k = atomicAdd(&counts[c], 1);
    src[cell_start[c] + k] = i;
  });
}

// 4. order each cell by atom id (rank sort inside the cell segment) and gather
//    the atom records into the sorted copies.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_gather(
    md_batch b, int mode, const int* cell_of, int* counts, const int* cell_start, const int* src,
    const double4* pos, const double* vel, const int* id, double4* pos_s, double* vel_s,
    int* id_s, const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const int n = b.n_atoms;
  FOR_ATOMS(b, slot, T, {
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
  });
}

// 5. copy the sorted records back and take them as the displacement reference.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_copyback(
    md_batch b, int mode, const double4* pos_s, const double* vel_s, const int* id_s,
    double4* pos, double* vel, int* id, double* pos_ref, const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const int n = b.n_atoms;
  FOR_ATOMS(b, i, T, {
    const double4 p = pos_s[i];
    pos[i] = p;
    vel[i] = vel_s[i];
    vel[n + i] = vel_s[n + i];
    vel[2 * n + i] = vel_s[2 * n + i];
    id[i] = id_s[i];
    pos_ref[i] = p.x;
    pos_ref[n + i] = p.y;
    pos_ref[2 * n + i] = p.z;
  });
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

// Candidates j of atom i in [jb, je) (cell order), 4 in flight; appends the
// neighbours in candidate order.
struct BuildCtx {
  double4 p;
  double len[3], inv[3];
  int per[3];
  double rns2;
  int i, cnt, max_neigh, lanes_log2, npad;
  int* neigh;
};

__device__ __forceinline__ void scan_range(BuildCtx& c, const double4* __restrict__ pos, int jb,
                                           int je) {
  const int lanes = 1 << c.lanes_log2;
  for (int j0 = jb; j0 < je; j0 += 4) {
    double4 q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = pos[min(j0 + u, je - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u;
      if (j >= je || j == c.i) continue;
      double dx = q[u].x - c.p.x, dy = q[u].y - c.p.y, dz = q[u].z - c.p.z;
      if (c.per[0]) dx = dx - c.len[0] * rint(dx * c.inv[0]);
      if (c.per[1]) dy = dy - c.len[1] * rint(dy * c.inv[1]);
      if (c.per[2]) dz = dz - c.len[2] * rint(dz * c.inv[2]);
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      if (r2 < c.rns2) {
        if (c.cnt < c.max_neigh)
          c.neigh[((size_t)(c.cnt >> c.lanes_log2) * c.npad + c.i) * lanes +
                  (c.cnt & (lanes - 1))] = j;
        ++c.cnt;
      }
    }
  }
}

__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_build(md_batch b, int mode,
                                                         const double4* __restrict__ pos,
                                                         const int* __restrict__ cell_start,
                                                         int* neigh, int* nneigh, int max_neigh,
                                                         int lanes_log2, int npad, double rns2,
                                                         md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  int wmax = 0, over = 0;
  FOR_ATOMS(b, i, T, {
    const md_domain& D = b.domains[T.rep];
    BuildCtx c;
    c.p = pos[i];
_Pragma("unroll")
    for (int a = 0; a < 3; ++a) {
      c.len[a] = D.len[a];
      c.inv[a] = D.inv_len[a];
      c.per[a] = D.periodic[a];
    }
    c.rns2 = rns2;
    c.i = i;
    c.cnt = 0;
    c.max_neigh = max_neigh;
    c.lanes_log2 = lanes_log2;
    c.npad = npad;
    c.neigh = neigh;
    const int cx = cell_coord(c.p.x, D.lo[0], D.inv_w[0], D.nc[0]);
    const int cy = cell_coord(c.p.y, D.lo[1], D.inv_w[1], D.nc[1]);
    const int cz = cell_coord(c.p.z, D.lo[2], D.inv_w[2], D.nc[2]);
    int sx[3], sy[3], sz[3];
    const int mx = stencil_axis(cx, D.nc[0], D.periodic[0], sx);
    const int my = stencil_axis(cy, D.nc[1], D.periodic[1], sy);
    const int mz = stencil_axis(cz, D.nc[2], D.periodic[2], sz);
    // Three z-neighbouring cells that do not wrap are one contiguous range.
    const bool zrun = (mz == 3) && (sz[0] + 1 == sz[1]) && (sz[1] + 1 == sz[2]);
    for (int ix = 0; ix < mx; ++ix)
      for (int iy = 0; iy < my; ++iy) {
        const int col = D.cell_off + (sx[ix] * D.nc[1] + sy[iy]) * D.nc[2];
        if (zrun) {
          scan_range(c, pos, cell_start[col + sz[0]], cell_start[col + sz[2] + 1]);
        } else {
          for (int iz = 0; iz < mz; ++iz)
            scan_range(c, pos, cell_start[col + sz[iz]], cell_start[col + sz[iz] + 1]);
        }
      }
    nneigh[i] = c.cnt < max_neigh ? c.cnt : max_neigh;
    over |= c.cnt > max_neigh;
    wmax = max(wmax, c.cnt);
  });
  if (__any(over)) {
    if ((threadIdx.x & (MD_WAVE - 1)) == 0) md_flag(ctl, MD_FLAG_NEIGH_OVERFLOW);
  }
  // One atomic per wavefront for the running maximum of the list length.
#pragma unroll
  for (int o = MD_WAVE / 2; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, MD_WAVE));
  if ((threadIdx.x & (MD_WAVE - 1)) == 0 && wmax > 0) atomicMax(&ctl->max_nneigh, wmax);
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
  const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
  MD_LAUNCH_TIMED(MD_KERNEL_BIN_COUNT, k_bin_count, grid, block, 0, st, *b, (int)mode,
                  (double4*)pos, cell_of, counts, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, b->n_cells, (int)mode, counts,
                     cell_start, c);
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
  const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
  MD_LAUNCH_TIMED(MD_KERNEL_BUILD, k_build, grid, block, 0, (hipStream_t)stream, *b, (int)mode,
                  (const double4*)pos, cell_start, nl->neigh, nl->nneigh, nl->max_neigh, lg,
                  md_npad(b->n_atoms), b->r_ns * b->r_ns, (md_ctl_dev*)ctl);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
