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
// Lanes below this one in mask m.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_count(md_batch b, int mode, double4* pos,
                                                             int* cell_of, int* rank_of,
                                                             int* counts, md_ctl_dev* ctl) {
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
    // Histogram with one atomic per run of equal cells among the wavefront's atoms
    // (they are still nearly in cell order from the last rebuild), all runs' atomics
    // in one instruction; each atom keeps the slot it got, so the scatter needs no
    // atomics.  Slot order inside a cell is arbitrary here; the gather ranks by id.
    // The active lanes of a tile are lanes 0 .. count - 1.
    const int lane = threadIdx.x & (MD_WAVE - 1);
    const int prev = __shfl(cell, lane > 0 ? lane - 1 : 0, MD_WAVE);
    const unsigned long long leads = __builtin_amdgcn_ballot_w64(lane == 0 || prev != cell);
    const int start = 63 - __builtin_clzll(leads & ((2ull << lane) - 1));  // this run's first lane
    int base = 0;
    if (lane == start) {
      const unsigned long long later = leads & ~((2ull << lane) - 1);
      const int end = later ? __builtin_ctzll(later) : T.count;
      base = atomicAdd(&counts[cell], end - lane);
    }
    base = __shfl(base, start, MD_WAVE);
    rank_of[i] = base + (lane - start);
  });
  if (bad) md_flag(ctl, bad);
}

// 2. exclusive scan of the histogram into cell_start (counts reset), over
// contiguous segments of cells, one 1024-thread block each: segment sums, one
// block scanning the sums, then each block scanning its segment from its offset.
__device__ __forceinline__ int block_incl_scan(int v, int* s_w, int& total) {
  const int lane = threadIdx.x & (MD_WAVE - 1), w = threadIdx.x / MD_WAVE;
  const int nw = blockDim.x / MD_WAVE;
#pragma unroll
  for (int o = 1; o < MD_WAVE; o <<= 1) {
    const int t = __shfl_up(v, o, MD_WAVE);
    if (lane >= o) v += t;
  }
  if (lane == MD_WAVE - 1) s_w[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int q = 0; q < nw; ++q) {
      const int t = s_w[q];
      s_w[q] = run;
      run += t;
    }
    s_w[16] = run;
  }
  __syncthreads();
  v += s_w[w];
  total = s_w[16];
  __syncthreads();  // s_w is reused by the next call
  return v;
}

// The whole histogram scan in one block, for grids of at most MD_SCAN_ONE_MAX cells: each
// thread scans a contiguous run of cells (one launch instead of three).
#define MD_SCAN_ONE_MAX 65536
__global__ __launch_bounds__(1024) void k_scan_one(int n_cells, int mode, int* counts,
                                                    int* cell_start, md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  __shared__ int s_w[17];
  const int per = (n_cells + 1023) / 1024;
  const int beg = min(n_cells, (int)threadIdx.x * per), end = min(n_cells, beg + per);
  int v = 0;
#pragma unroll 8
  for (int k = beg; k < end; ++k) v += counts[k];
  int total;
  int run = block_incl_scan(v, s_w, total) - v;
#pragma unroll 8
  for (int k = beg; k < end; ++k) {
    const int c = counts[k];
    cell_start[k] = run;
    run += c;
    counts[k] = 0;
  }
  if (threadIdx.x == 0) {
    cell_start[n_cells] = total;
    ctl->n_rebuilds += 1;
  }
}

__global__ __launch_bounds__(1024) void k_scan_sums(int n_cells, int seg, int mode,
                                                     const int* counts, int* bsum,
                                                     md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  __shared__ int s_w[17];
  const int beg = blockIdx.x * seg, end = min(n_cells, beg + seg);
  int v = 0;
  for (int k = beg + threadIdx.x; k < end; k += blockDim.x) v += counts[k];
  int total;
  block_incl_scan(v, s_w, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int nb, int n_cells, int mode, int* bsum,
                                                    int* cell_start, md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  __shared__ int s_w[17];
  const int t = threadIdx.x;
  const int v = t < nb ? bsum[t] : 0;
  int total;
  const int incl = block_incl_scan(v, s_w, total);
  if (t < nb) bsum[t] = incl - v;
  if (t == 0) {
    cell_start[n_cells] = total;
    ctl->n_rebuilds += 1;
  }
}

__global__ __launch_bounds__(1024) void k_scan_apply(int n_cells, int seg, int mode, int* counts,
                                                      const int* bsum, int* cell_start,
                                                      md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  __shared__ int s_w[17];
  const int beg = blockIdx.x * seg, end = min(n_cells, beg + seg);
  int carry = bsum[blockIdx.x];
  for (int c0 = beg; c0 < end; c0 += blockDim.x) {
    const int k = c0 + threadIdx.x;
    const int v = k < end ? counts[k] : 0;
    int total;
    const int incl = block_incl_scan(v, s_w, total);
    if (k < end) {
      cell_start[k] = carry + incl - v;
      counts[k] = 0;
    }
    carry += total;
  }
}

// 3. scatter atom indices (and their ids) into their cell segments, at the slots
//    the histogram handed out.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_scatter(md_batch b, int mode,
                                                               const int* cell_of,
                                                               const int* rank_of,
                                                               const int* cell_start,
                                                               const int* id, int* src, int* sid,
                                                               const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  FOR_ATOMS(b, i, T, {
    const int dst = cell_start[cell_of[i]] + rank_of[i];
    src[dst] = i;
    sid[dst] = id[i];
  });
}

// 4. order each cell by atom id (rank sort inside the cell segment) and gather
//    the atom records into the sorted copies.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_gather(
    md_batch b, int mode, const int* cell_of, const int* cell_start, const int* src,
    const int* sid, const double4* pos, const double* vel, double4* pos_s, double* vel_s,
    int* id_s, const md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const int n = b.n_atoms;
  FOR_ATOMS(b, slot, T, {
    const int a = src[slot];
    const int c = cell_of[a];
    const int beg = cell_start[c], end = cell_start[c + 1];
    const int my = sid[slot];
    int rank = 0;  // ids are unique: the rank by id is a permutation of the segment
    for (int k = beg; k < end; ++k) rank += sid[k] < my;
    const int dst = beg + rank;
    pos_s[dst] = pos[a];
    vel_s[dst] = vel[a];
    vel_s[n + dst] = vel[n + a];
    vel_s[2 * n + dst] = vel[2 * n + a];
    id_s[dst] = my;
  });
}

// 5. copy the sorted records back and take them as the displacement reference.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bin_copyback(
    md_batch b, int mode, const double4* pos_s, const double* vel_s, const int* id_s,
    double4* pos, double* vel, int* id, double* pos_ref, md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  const int n = b.n_atoms;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->n_dmax = 0;      // displacements now measured afresh
    ctl->rec_stale = 1;   // atoms reordered: carried-over neighbour records are void
  }
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
// Verlet list (Sec. 1.4): the candidates of every atom of a cell are the atoms of
// the (de-duplicated) 3x3x3 block of cells around it, the same set for all atoms
// of the cell.  One wavefront takes one cell: its lanes hold 64 candidates at a
// time (positions in registers, loaded once per cell rather than once per atom)
// and test them against each atom of the cell in turn; a ballot of the accepted
// lanes gives every accepted candidate its slot, so the list is written in
// candidate order (stencil cell order, then cell order) in a single pass.
// ---------------------------------------------------------------------------
constexpr int CW = 4;                  // wavefronts (cells) per block
constexpr int CELL_BLOCK = CW * MD_WAVE;

// Stencil cell t (0..2) along one axis for an atom in cell c: the cell index, or -1
// when there is none (outside a non-periodic box, or a duplicate when nc < 3), and
// the image k = rint(d / L) that a candidate in it has (d = x_j - x_i): +1 for a
// cell reached by wrapping below 0, -1 by wrapping above nc - 1.
__device__ __forceinline__ int stencil_cell(int c, int t, int nc, int periodic, int& k) {
  k = 0;
  if (periodic && nc < 3) return t < nc ? t : -1;
  int q = c + t - 1;
  if (q < 0) {
    if (!periodic) return -1;
    q += nc;
    k = 1;
  } else if (q >= nc) {
    if (!periodic) return -1;
    q -= nc;
    k = -1;
  }
  return q;
}

// Test modes: PLAIN for a cell whose block does not wrap (d itself is the minimum
// image: |d| < 2 w <= 2 L / 5 < L / 2 when nc >= 5), SHIFT for a wrapping block
// with nc >= 5 on every periodic axis (the image of each stencil cell is fixed, so
// d - L k is the minimum image, the same operations as d - L rint(d / L)), RINT
// for small grids (nc < 5 on a periodic axis): the minimum image per candidate.
enum { PLAIN = 0, SHIFT = 1, RINT = 2 };

struct Cand {
  double x, y, z;     // candidate position
  double sx, sy, sz;  // L k per axis (SHIFT)
  int j;              // candidate index
  bool valid;
};

// Entry `slot` of atom ia: row slot / lanes, column ia * lanes + slot % lanes.
// FAST: the whole list spans < 4 GiB and a row < 2^24 ints, so a 32-bit byte offset
// from the atom's (wave-uniform) first entry addresses it.
template <bool FAST>
__device__ __forceinline__ int* entry(int* neigh, int ia, int slot, int lanes_log2,
                                      unsigned row) {
  const int lanes = 1 << lanes_log2;
  int* at = neigh + (size_t)ia * lanes;
  const unsigned q = (unsigned)slot >> lanes_log2, col = (unsigned)slot & (lanes - 1);
  return FAST ? (int*)((char*)at + ((__umul24(q, row) + col) << 2)) : at + ((size_t)q * row + col);
}


// Candidate c against atom k of the cell (position in s_p, index ia).
template <int MODE>
__device__ __forceinline__ bool accept_pair(const Cand& c, double (*s_p)[MD_WAVE], int k, int ia,
                                            const double* len, const double* inv, const int* per,
                                            double rns2) {
  double dx = c.x - s_p[0][k], dy = c.y - s_p[1][k], dz = c.z - s_p[2][k];
  if (MODE == SHIFT) {
    dx = dx - c.sx;
    dy = dy - c.sy;
    dz = dz - c.sz;
  } else if (MODE == RINT) {
    if (per[0]) dx = dx - len[0] * rint(dx * inv[0]);
    if (per[1]) dy = dy - len[1] * rint(dy * inv[1]);
    if (per[2]) dz = dz - len[2] * rint(dz * inv[2]);
  }
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  return c.valid & (c.j != ia) & (r2 < rns2);
}

template <int MODE, bool FAST>
__device__ __forceinline__ void cell_lists(const md_domain& D, int a0, int na, int C,
                                           const int* s_beg, const int* s_start,
                                           const int* s_code, double (*s_p)[MD_WAVE],
                                           const double4* __restrict__ pos, int* neigh,
                                           int* nneigh, int max_neigh, int lanes_log2, int npad,
                                           double rns2, bool img, md_ctl_dev* ctl) {
  const int lane = threadIdx.x & (MD_WAVE - 1);
  const int lanes = 1 << lanes_log2;
  const unsigned row = (unsigned)npad * lanes;  // ints per list row
  double len[3], inv[3];
  int per[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    len[q] = D.len[q];
    inv[q] = D.inv_len[q];
    per[q] = D.periodic[q];
  }
  // candidate v of the flattened stencil: range r = the last with s_beg[r] <= v
  auto make = [&](int v) {
    Cand c;
    c.valid = v < C;
    int r = 0;
#pragma unroll
    for (int st = 16; st > 0; st >>= 1)
      if (s_beg[r + st] <= v) r += st;
    c.j = c.valid ? s_start[r] + (v - s_beg[r]) : a0;
    const double4 q = pos[c.j];
    c.x = q.x;
    c.y = q.y;
    c.z = q.z;
    const int code = s_code[r];
    const int kx = (code & 3) - 1, ky = ((code >> 2) & 3) - 1, kz = ((code >> 4) & 3) - 1;
    c.sx = kx == 0 ? 0.0 : (kx > 0 ? len[0] : -len[0]);
    c.sy = ky == 0 ? 0.0 : (ky > 0 ? len[1] : -len[1]);
    c.sz = kz == 0 ? 0.0 : (kz > 0 ? len[2] : -len[2]);
    return c;
  };
  int over = 0, most = 0;
  for (int g0 = 0; g0 < na; g0 += MD_WAVE) {
    const int gc = min(MD_WAVE, na - g0);
    if (lane < gc) {
      const double4 q = pos[a0 + g0 + lane];
      s_p[0][lane] = q.x;
      s_p[1][lane] = q.y;
      s_p[2][lane] = q.z;
    }
    __builtin_amdgcn_wave_barrier();
    int tot = 0;  // lane k: accepted candidates of atom g0 + k so far
    Cand nx = make(lane);
    for (int v0 = 0; v0 < C; v0 += MD_WAVE) {
      const Cand c = nx;
      if (v0 + MD_WAVE < C) nx = make(v0 + MD_WAVE + lane);  // next chunk in flight
      // two atoms per trip: their distance chains overlap
      for (int k = 0; k < gc; k += 2) {
        const int k1 = min(k + 1, gc - 1);  // gc odd: the last trip tests atom k twice
        const bool ok0 = accept_pair<MODE>(c, s_p, k, a0 + g0 + k, len, inv, per, rns2);
        const bool ok1 = accept_pair<MODE>(c, s_p, k1, a0 + g0 + k1, len, inv, per, rns2) &&
                         k1 != k;
        const unsigned long long m0 = __builtin_amdgcn_ballot_w64(ok0);
        const unsigned long long m1 = __builtin_amdgcn_ballot_w64(ok1);
        const int base0 = __builtin_amdgcn_readlane(tot, k);
        const int base1 = __builtin_amdgcn_readlane(tot, k1);
        const int slot0 = base0 + lanes_below(m0), slot1 = base1 + lanes_below(m1);
        if (ok0 && slot0 < max_neigh)
          *entry<FAST>(neigh, a0 + g0 + k, slot0, lanes_log2, row) = c.j;
        if (ok1 && slot1 < max_neigh)
          *entry<FAST>(neigh, a0 + g0 + k1, slot1, lanes_log2, row) = c.j;
        tot = lane == k ? base0 + (int)__popcll(m0) : tot;
        tot = lane == k1 && k1 != k ? base1 + (int)__popcll(m1) : tot;
      }
    }
    if (lane < gc) {
      nneigh[a0 + g0 + lane] = (tot < max_neigh ? tot : max_neigh) | (img ? MD_NN_IMG : 0);
      over |= tot > max_neigh;
      most = max(most, tot);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (__any(over)) {
    if (lane == 0) md_flag(ctl, MD_FLAG_NEIGH_OVERFLOW);
  }
#pragma unroll
  for (int o = MD_WAVE / 2; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o, MD_WAVE));
  if (lane == 0 && most > 0) atomicMax(&ctl->max_nneigh, most);
}

__global__ __launch_bounds__(CELL_BLOCK) void k_build(md_batch b, int mode,
                                                      const double4* __restrict__ pos,
                                                      const int* __restrict__ cell_start,
                                                      int* neigh, int* nneigh, int max_neigh,
                                                      int lanes_log2, int npad, double rns2,
                                                      md_ctl_dev* ctl) {
  if (skip_rebuild(mode, ctl)) return;
  __shared__ int s_beg[CW][33], s_start[CW][32], s_code[CW][32];
  __shared__ double s_p[CW][3][MD_WAVE];
  const int w = threadIdx.x / MD_WAVE, lane = threadIdx.x & (MD_WAVE - 1);
  const int cell = md_remap_block((b.n_cells + CW - 1) / CW) * CW + w;
  if (cell >= b.n_cells) return;  // whole wavefronts only
  // the box of this cell: the last domain whose cells start at or before it
  int lo = 0, hi = b.n_rep - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.domains[mid].cell_off <= cell) lo = mid; else hi = mid - 1;
  }
  const md_domain& D = b.domains[lo];
  const int a0 = __builtin_amdgcn_readfirstlane(cell_start[cell]);
  const int na = __builtin_amdgcn_readfirstlane(cell_start[cell + 1]) - a0;
  if (na == 0) return;
  const int local = cell - D.cell_off;
  const int c2 = local % D.nc[2], c1 = (local / D.nc[2]) % D.nc[1], c0 = local / (D.nc[2] * D.nc[1]);
  // lane t < 27 takes stencil cell (t / 9, t / 3 % 3, t % 3): its atom range and image
  int cnt = 0, start = 0, code = 0;
  if (lane < 27) {
    int kx, ky, kz;
    const int qx = stencil_cell(c0, lane / 9, D.nc[0], D.periodic[0], kx);
    const int qy = stencil_cell(c1, (lane / 3) % 3, D.nc[1], D.periodic[1], ky);
    const int qz = stencil_cell(c2, lane % 3, D.nc[2], D.periodic[2], kz);
    if (qx >= 0 && qy >= 0 && qz >= 0) {
      const int q = D.cell_off + (qx * D.nc[1] + qy) * D.nc[2] + qz;
      start = cell_start[q];
      cnt = cell_start[q + 1] - start;
      code = (kx + 1) | ((ky + 1) << 2) | ((kz + 1) << 4);
    }
  }
  // exclusive prefix of the range sizes over the lanes
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const int u = __shfl_up(incl, o, MD_WAVE);
    if (lane >= o) incl += u;
  }
  const int C = __builtin_amdgcn_readlane(incl, 31);
  if (lane < 32) {
    s_beg[w][lane] = lane < 27 ? incl - cnt : C;
    s_start[w][lane] = start;
    s_code[w][lane] = code;
  }
  if (lane == 0) s_beg[w][32] = C;
  __builtin_amdgcn_wave_barrier();
  // the block wraps (image flag for the force passes), and the test mode
  bool img = false, small = false;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int cq = q == 0 ? c0 : (q == 1 ? c1 : c2);
    if (D.periodic[q]) {
      img |= (D.nc[q] < 3) || cq == 0 || cq == D.nc[q] - 1;
      small |= D.nc[q] < 5;
    }
  }
  const bool fast = ((size_t)npad << lanes_log2) < ((size_t)1 << 24) &&
                    (size_t)max_neigh * npad * sizeof(int) < ((size_t)1 << 32);
  const int mode_ = small ? RINT : (img ? SHIFT : PLAIN);
#define MD_CELL_LISTS(M, R24)                                                                   \
  cell_lists<M, R24>(D, a0, na, C, s_beg[w], s_start[w], s_code[w], s_p[w], pos, neigh, nneigh, \
                     max_neigh, lanes_log2, npad, rns2, img, ctl)
  if (fast) {
    if (mode_ == PLAIN) MD_CELL_LISTS(PLAIN, true);
    else if (mode_ == SHIFT) MD_CELL_LISTS(SHIFT, true);
    else MD_CELL_LISTS(RINT, true);
  } else {
    if (mode_ == PLAIN) MD_CELL_LISTS(PLAIN, false);
    else if (mode_ == SHIFT) MD_CELL_LISTS(SHIFT, false);
    else MD_CELL_LISTS(RINT, false);
  }
#undef MD_CELL_LISTS
}

}  // namespace

extern "C" int md_bin_cells(const md_batch* b, md_rebuild_mode mode, double* pos, double* vel,
                            int* id, double* pos_ref, int* cell_start, void* ws, void* ctl,
                            void* stream) {
  if (!md_batch_ok(b) || !pos || !vel || !id || !pos_ref || !cell_start || !ws || !ctl)
    return MD_ERR_ARG;
  if (mode != MD_ALWAYS && mode != MD_IF_FLAGGED) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  const md_ws_layout L = md_ws_plan(b);
  char* w = (char*)ws;
  int* cell_of = (int*)(w + L.cell_of);
  int* rank_of = (int*)(w + L.rank);
  int* src = (int*)(w + L.src);
  int* sid = (int*)(w + L.sid);
  int* counts = (int*)(w + L.counts);
  double4* pos_s = (double4*)(w + L.pos_s);
  double* vel_s = (double*)(w + L.vel_s);
  int* id_s = (int*)(w + L.id_s);
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
  MD_LAUNCH_TIMED(MD_KERNEL_BIN_COUNT, k_bin_count, grid, block, 0, st, *b, (int)mode,
                  (double4*)pos, cell_of, rank_of, counts, c);
  MD_LAUNCH_CHECK();
  if (b->n_cells <= MD_SCAN_ONE_MAX) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(1024), 0, st, b->n_cells, (int)mode, counts,
                       cell_start, c);
    MD_LAUNCH_CHECK();
  } else {
    const int nb = std::min(MD_SCAN_BLOCKS, (b->n_cells + 1023) / 1024);
    const int seg = (b->n_cells + nb - 1) / nb;
    int* bsum = (int*)(w + L.scan);
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, st, b->n_cells, seg, (int)mode,
                       counts, bsum, c);
    MD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, nb, b->n_cells, (int)mode, bsum,
                       cell_start, c);
    MD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, st, b->n_cells, seg, (int)mode,
                       counts, bsum, cell_start, c);
    MD_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_bin_scatter, grid, block, 0, st, *b, (int)mode, cell_of, rank_of,
                     cell_start, id, src, sid, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_gather, grid, block, 0, st, *b, (int)mode, cell_of, cell_start, src,
                     sid, (const double4*)pos, vel, pos_s, vel_s, id_s, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_copyback, grid, block, 0, st, *b, (int)mode, pos_s, vel_s, id_s,
                     (double4*)pos, vel, id, pos_ref, c);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" int md_build_neighbors(const md_batch* b, md_rebuild_mode mode, const double* pos,
                                  const int* cell_start, const md_nlist* nl, void* ctl,
                                  void* stream) {
  if (!md_batch_ok(b) || !pos || !cell_start || !nl || !nl->neigh || !nl->nneigh || !ctl)
    return MD_ERR_ARG;
  if (mode != MD_ALWAYS && mode != MD_IF_FLAGGED) return MD_ERR_ARG;
  int lg = -1;
  for (int k = 0; k <= 4; ++k)
    if (nl->lanes == (1 << k)) lg = k;
  if (lg < 0 || nl->max_neigh < nl->lanes || nl->max_neigh % nl->lanes) return MD_ERR_ARG;
  if (!(b->r_ns > 0.0)) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  const dim3 grid(md_grid_blocks((b->n_cells + CW - 1) / CW)), block(CELL_BLOCK);
  MD_LAUNCH_TIMED(MD_KERNEL_BUILD, k_build, grid, block, 0, (hipStream_t)stream, *b, (int)mode,
                  (const double4*)pos, cell_start, nl->neigh, nl->nneigh, nl->max_neigh, lg,
                  md_npad(b->n_atoms), b->r_ns * b->r_ns, (md_ctl_dev*)ctl);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
