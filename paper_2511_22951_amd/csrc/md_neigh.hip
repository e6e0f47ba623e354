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
  // The rebuild decision: every block reduces the displacement maxima of the last
  // drift itself (no cross-block communication); block 0 publishes it for the
  // other rebuild kernels of this call.
  const bool go = mode == MD_ALWAYS || md_displacement_exceeded(ctl);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->rebuild = go ? 1 : 0;
  if (!go) return;
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
    double4* pos, double* vel, int* id, double* pos_ref, md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const int n = b.n_atoms;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->n_dmax = 0;  // displacements now measured afresh
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

// Verlet list with BL lanes per atom.  The atom's candidates are the atoms of the
// (de-duplicated) 3x3x3 cell block, taken as up to 27 index ranges (three
// z-neighbouring cells that do not wrap form one range).  The atom's BL lanes
// walk each range in lock step, BL consecutive candidates per round; a wavefront
// ballot of the accepted flags gives every accepted candidate its slot (the
// number of accepted candidates before it), so one pass writes the list in
// candidate order: deterministic, and neighbouring atoms get similar lists.
// The tile's 64 lists are assembled in LDS and written out row by row, each
// row of the strided layout being one contiguous segment (coalesced stores).
constexpr int BL = 8;
constexpr int BU = 4;                  // candidate rounds per trip (loads in flight)
constexpr int BUILD_BLOCK = 64 * BL;  // one work tile per block
constexpr int MAX_STAGED = 192;       // 64 lists of this length + ranges fit 64 KB of LDS


// r^2 < r_ns^2 for the pair, with the minimum image when IMG.  Without it the
// result is identical: for an atom whose cell block does not wrap, |d| < L/2 and
// d - L rint(d / L) = d - 0 = d exactly.
template <bool IMG>
__device__ __forceinline__ bool accept(const double4& p, const double4& q, const double* len,
                                       const double* inv, const int* per, double rns2) {
  double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
  if (IMG) {
    if (per[0]) dx = dx - len[0] * rint(dx * inv[0]);
    if (per[1]) dy = dy - len[1] * rint(dy * inv[1]);
    if (per[2]) dz = dz - len[2] * rint(dz * inv[2]);
  }
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  return r2 < rns2;
}

template <bool STAGE>
__global__ __launch_bounds__(BUILD_BLOCK) void k_build(md_batch b, int mode,
                                                       const double4* __restrict__ pos,
                                                       const int* __restrict__ cell_start,
                                                       int* neigh, int* nneigh, int max_neigh,
                                                       int lanes_log2, int npad, double rns2,
                                                       md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;
  const md_tile T = b.tiles[t];
  const md_domain& D = b.domains[T.rep];
  const int a = threadIdx.x / BL, l = threadIdx.x % BL;
  const bool active = a < T.count;
  const int i = T.first + (active ? a : 0);
  double len[3], inv[3];
  int per[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    len[q] = D.len[q];
    inv[q] = D.inv_len[q];
    per[q] = D.periodic[q];
  }
  const double4 p = pos[i];
  const int cx = cell_coord(p.x, D.lo[0], D.inv_w[0], D.nc[0]);
  const int cy = cell_coord(p.y, D.lo[1], D.inv_w[1], D.nc[1]);
  const int cz = cell_coord(p.z, D.lo[2], D.inv_w[2], D.nc[2]);
  int sx[3], sy[3], sz[3];
  const int mx = stencil_axis(cx, D.nc[0], D.periodic[0], sx);
  const int my = stencil_axis(cy, D.nc[1], D.periodic[1], sy);
  const int mz = stencil_axis(cz, D.nc[2], D.periodic[2], sz);
  const bool zrun = (mz == 3) && (sz[0] + 1 == sz[1]) && (sz[1] + 1 == sz[2]);
  // the atom's candidate ranges, shared by its lanes through LDS; the (x, y)
  // columns of the stencil are spread over the atom's lanes so that their
  // cell_start lookups are in flight together
  __shared__ int2 s_rng[64][27];
  __shared__ int s_nr[64];
  {
    const int ncol = mx * my, per_col = zrun ? 1 : mz;
    for (int c = l; c < ncol; c += BL) {
      const int ix = c / my, iy = c - ix * my;
      const int col = D.cell_off + (sx[ix] * D.nc[1] + sy[iy]) * D.nc[2];
      if (zrun) {
        s_rng[a][c] = make_int2(cell_start[col + sz[0]], cell_start[col + sz[2] + 1]);
      } else {
        for (int iz = 0; iz < mz; ++iz)
          s_rng[a][c * mz + iz] = make_int2(cell_start[col + sz[iz]], cell_start[col + sz[iz] + 1]);
      }
    }
    if (l == 0) s_nr[a] = active ? ncol * per_col : 0;
  }
  __syncthreads();
  const int nrng = s_nr[a];
  extern __shared__ int s_list[];  // [64][max_neigh]
  bool img = false;
  if (D.periodic[0]) img |= (D.nc[0] < 3) || cx == 0 || cx == D.nc[0] - 1;
  if (D.periodic[1]) img |= (D.nc[1] < 3) || cy == 0 || cy == D.nc[1] - 1;
  if (D.periodic[2]) img |= (D.nc[2] < 3) || cz == 0 || cz == D.nc[2] - 1;
  // the minimum-image test is taken by the whole wavefront when any of its atoms
  // needs it (for the others it gives the identical result)
  const bool wimg = __any(img);
  const int lanes = 1 << lanes_log2;
  const int gshift = (threadIdx.x & (MD_WAVE - 1)) & ~(BL - 1);  // the atom's lanes in the ballot
  const unsigned below = (1u << l) - 1u;
  int total = 0;
  for (int r = 0; r < nrng; ++r) {
    const int jb = s_rng[a][r].x, je = s_rng[a][r].y;
    // BU rounds of BL candidates per trip, their loads issued together
    for (int j0 = jb; j0 < je; j0 += BL * BU) {
      double4 q[BU];
#pragma unroll
      for (int u = 0; u < BU; ++u) q[u] = pos[min(j0 + u * BL + l, je - 1)];
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        const int j = j0 + u * BL + l;
        const bool in = wimg ? accept<true>(p, q[u], len, inv, per, rns2)
                             : accept<false>(p, q[u], len, inv, per, rns2);
        const bool ok = (j < je) & (j != i) & in;
        const unsigned g = (unsigned)(__ballot(ok) >> gshift) & ((1u << BL) - 1u);
        if (ok) {
          const int slot = total + __popc(g & below);
          if (slot < max_neigh) {
            if (STAGE)
              s_list[a * max_neigh + slot] = j;
            else
              neigh[((size_t)(slot >> lanes_log2) * npad + i) * lanes + (slot & (lanes - 1))] = j;
          }
        }
        total += __popc(g);
      }
    }
  }
  if (STAGE) {
    // coalesced write-out: row q of the layout holds entries q*lanes .. q*lanes+lanes-1
    // of every atom; the tile's atoms occupy 64*lanes consecutive ints of each row.
    __shared__ int s_cnt[64];
    if (l == 0) s_cnt[a] = active ? min(total, max_neigh) : 0;
    __syncthreads();
    int tmax = 0;
    for (int q = 0; q < 64; ++q) tmax = max(tmax, s_cnt[q]);
    const int rows = (tmax + lanes - 1) >> lanes_log2;
    const int span = 64 * lanes;
    for (int e = threadIdx.x; e < rows * span; e += blockDim.x) {
      const int q = e / span, w = e - q * span;
      const int aa = w >> lanes_log2, m = q * lanes + (w & (lanes - 1));
      if (aa < T.count && m < s_cnt[aa])
        neigh[((size_t)q * npad + T.first) * lanes + w] = s_list[aa * max_neigh + m];
    }
  }
  int over = 0, wmax = 0;
  if (active && l == 0) {
    // img: the stencil crosses a periodic boundary (wrapped cell, or fewer than 3 cells)
    nneigh[i] = (total < max_neigh ? total : max_neigh) | (img ? MD_NN_IMG : 0);
    over = total > max_neigh;
    wmax = total;
  }
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
  const dim3 grid(md_grid_blocks(b->n_tiles)), block(BUILD_BLOCK);
  // Lists are staged in LDS (coalesced write-out) when the tile's 64 lists fit
  // beside the static ranges within 64 KB; longer lists are stored directly.
  const size_t lds = (size_t)64 * nl->max_neigh * sizeof(int);
  if (nl->max_neigh <= MAX_STAGED)
    MD_LAUNCH_TIMED(MD_KERNEL_BUILD, k_build<true>, grid, block, lds, (hipStream_t)stream, *b,
                    (int)mode, (const double4*)pos, cell_start, nl->neigh, nl->nneigh,
                    nl->max_neigh, lg, md_npad(b->n_atoms), b->r_ns * b->r_ns,
                    (md_ctl_dev*)ctl);
  else
    MD_LAUNCH_TIMED(MD_KERNEL_BUILD, k_build<false>, grid, block, 0, (hipStream_t)stream, *b,
                    (int)mode, (const double4*)pos, cell_start, nl->neigh, nl->nneigh,
                    nl->max_neigh, lg, md_npad(b->n_atoms), b->r_ns * b->r_ns,
                    (md_ctl_dev*)ctl);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
