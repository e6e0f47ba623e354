// Adjoint of the EAM forces with respect to the spline coefficients.
//
// For a cotangent G_i = dL/dF_i and fixed positions, dL/dc = -dD/dc with
// D = sum_i G_i . grad_i E (since F_i = -grad_i E).  Writing the EAM gradient
// (Sec. 1.6) pair by pair and symmetrising over the full list, with
// u_ij = r_ij / r_ij, s_ij = (G_i - G_j) . u_ij and tau_i = sum_j rho'(r_ij) s_ij:
//   D = 1/2 sum_{i != j} phi'(r_ij) s_ij + sum_i F'(rhobar_i) tau_i.
// Differentiating with respect to the coefficients of the three B-splines
// (beta_k the basis function of coefficient k):
//   dD/dc_phi_k = 1/2 sum_{i,j} beta_k'(r_ij) s_ij
//   dD/dc_rho_k = sum_{i,j} F'_i beta_k'(r_ij) s_ij + sum_i F''_i tau_i sum_j beta_k(r_ij)
//   dD/dc_F_k   = sum_i beta_k'(rhobar_i) tau_i
// The F'' and beta' terms are the mixed second derivatives.
//
// One kernel visits each atom's list twice (the second visit needs the complete
// tau_i); where the density Jacobian sum_j beta_k(r_ij) = d rhobar_i / d c_rho_k of
// the fixed positions is kept, the second visit is a product with its rows instead.
// The same file holds that Jacobian's kernel and the force-matching loss.  Each
// wavefront accumulates into its own LDS bins; a block adds its wavefronts' bins in
// wave order into per-tile partials, and a second kernel adds the tile partials in
// a fixed order.  All sums are FP64.  Pair distances crowd
// around the neighbour shells, so many lanes of one atomic add hit the same phi or
// rho bin and the LDS serialises them: each wavefront keeps several copies of those
// bins (lane l adds into copy l mod copies), laid out to start on different banks.
#include <math.h>

#include "md_internal.h"

namespace {

#define MD_ADJ_MAX_BINS 1024
#define MD_ADJ_U 2        // list entries in flight per lane
#define MD_ADJ_COPIES 8   // most copies of the phi and rho bins per wavefront
#define MD_ADJ_COPIES_JAC 4  // the same with the density Jacobian (fewer adds per pair)
#define MD_ADJ_LDS 49152  // LDS per block that the copies may fill
#define MD_JAC_MAX_COEF 128  // density Jacobian: rows of 64 atoms in LDS (64 KiB)

__device__ __forceinline__ void bspline_basis(double t, double b[4], double g[4]) {
  const double s = 1.0 - t;
  b[0] = s * s * s / 6.0;
  b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  b[3] = t * t * t / 6.0;
  g[0] = -0.5 * s * s;
  g[1] = 0.5 * (3.0 * t * t - 4.0 * t);
  g[2] = 0.5 * (-3.0 * t * t + 2.0 * t + 1.0);
  g[3] = 0.5 * t * t;
}

__device__ __forceinline__ int interval(double x, double lo, double inv_h, int nint, double& t,
                                        bool& oor) {
  const double u = (x - lo) * inv_h;
  if (u < 0.0 || u > (double)nint) oor = true;
  double f = floor(u);
  if (f < 0.0) f = 0.0;
  if (f > (double)(nint - 1)) f = (double)(nint - 1);
  t = u - f;
  return (int)f;
}

struct AdjGeom {
  const double* c_rho;
  double r_lo, r_inv_h, e_lo, e_inv_h;
  int nr, ne;           // intervals
  int n_phi, n_rho, n_emb, n_bins;
  int copies, stride;   // copies of a wavefront's phi|rho bins, doubles from one to the next
};

// 1/sqrt(x) for a normal x > 0: the hardware estimate (about 23 correct bits) refined
// by two Newton-Raphson steps y <- y + y (1/2 - x y^2 / 2), each of which roughly
// doubles the correct bits.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-hx * y, y, 0.5), y);
  return y;
}

// Interval of x on a uniform grid without the range check: t in [0, 1] inside the
// clamped interval k (the first visit records the range of u).
__device__ __forceinline__ int interval_u(double u, int nint, double& t) {
  const double f = fmin(fmax(floor(u), 0.0), (double)(nint - 1));
  t = u - f;
  return (int)f;
}

// Per-lane list visit with the indices of the next U entries loaded while the
// records of the current U are in flight (one round trip per U entries).  Entry m
// of the lane sits U-wise at nb + m * stride; padding past the lane's cnt entries
// loads the atom itself and is not visited.
template <int U, typename Load, typename Pair>
__device__ __forceinline__ void adj_visit(const int* nb, size_t stride, int cnt, int self,
                                          Load load, Pair pair) {
  if (cnt <= 0) return;
  int jn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) jn[u] = nb[u < cnt ? u * stride : 0];
  for (int b0 = 0; b0 < cnt; b0 += U) {
    decltype(load(0)) q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = load(b0 + u < cnt ? jn[u] : self);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = b0 + U + u;
      jn[u] = nb[m < cnt ? m * stride : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (b0 + u < cnt) pair(q[u]);
  }
}

struct AdjRec1 {
  double x, y, z, gx, gy, gz;
};

// Minimum-image separation d = x_j - x_i (a non-periodic axis has inv = 0, so its
// shift is 0) and its square, with the multiply-adds written out so that every
// kernel decides r < r_c on the same bits.
__device__ __forceinline__ double pair_disp2(const double4& pi, double x, double y, double z,
                                             const double len[3], const double inv[3],
                                             double d[3]) {
  d[0] = x - pi.x;
  d[1] = y - pi.y;
  d[2] = z - pi.z;
#pragma unroll
  for (int q = 0; q < 3; ++q) d[q] = fma(-len[q], rint(d[q] * inv[q]), d[q]);
  return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

// 6 beta_{k+q}(t), q = 0..3, of the cubic B-spline on the interval's local t.
__device__ __forceinline__ void basis6(double tt, double bb[4]) {
  const double t2 = tt * tt, s = 1.0 - tt;
  bb[0] = s * s * s;
  bb[1] = fma(t2, fma(3.0, tt, -6.0), 4.0);
  bb[2] = fma(tt, fma(tt, fma(-3.0, tt, 3.0), 3.0), 1.0);
  bb[3] = t2 * tt;
}

// Per pair the basis enters through fixed multiples that are taken out of the
// loops: 2 beta'_k(t) / h (the factor 1/2 and 1/h go into the per-atom weights) in
// the first visit and 6 beta_k(t) (the 1/6 goes into c_F'') in the second.
// JAC: the second visit is replaced by the density Jacobian of the atoms
// (jac[i][k] = d rhobar_i / d c_rho_k, fixed positions): its F'' term,
// sum_i F''_i tau_i jac[i][k], is one product of the tile's rows with the weights
// -F''_i tau_i, wave w taking atoms w, w + waves, ... in order.
template <int LANES, int U, bool JAC>
__global__ __launch_bounds__(64 * LANES) void k_eam_adjoint(
    md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, const double* __restrict__ saved,
    const double* __restrict__ jac, const double* __restrict__ G, AdjGeom g, double rc2,
    double* tile_bins, md_ctl_dev* ctl) {
  // LDS: phi|rho bins [waves][copies][stride], F bins [waves][n_emb], rho coefficients,
  // and (JAC) the tile's per-atom weights
  extern __shared__ double bins[];
  const int nw = blockDim.x / MD_WAVE, wid = threadIdx.x / MD_WAVE;
  const int n_hot = g.n_phi + g.n_rho, n_copy = nw * g.copies;
  double* emb_bins = bins + (size_t)n_copy * g.stride;
  double* c_rho = emb_bins + (size_t)nw * g.n_emb;
  double* s_w = c_rho + g.n_rho;  // [64] (JAC)
  for (int q = threadIdx.x; q < n_copy * g.stride + nw * g.n_emb; q += blockDim.x) bins[q] = 0.0;
  for (int q = threadIdx.x; q < g.n_rho; q += blockDim.x) c_rho[q] = g.c_rho[q];
  __syncthreads();
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;
  double* b_phi = bins + ((size_t)wid * g.copies + (threadIdx.x & (g.copies - 1))) * g.stride;
  double* b_rho = b_phi + g.n_phi;
  double* b_emb = emb_bins + (size_t)wid * g.n_emb;
  const md_tile T = b.tiles[t];
  const md_domain& Dm = b.domains[T.rep];
  // minimum image: a non-periodic axis gets 0 as inverse length (its shift is 0)
  const double len[3] = {Dm.len[0], Dm.len[1], Dm.len[2]};
  const double inv[3] = {Dm.periodic[0] ? Dm.inv_len[0] : 0.0,
                         Dm.periodic[1] ? Dm.inv_len[1] : 0.0,
                         Dm.periodic[2] ? Dm.inv_len[2] : 0.0};
  const int a = threadIdx.x / LANES, l = threadIdx.x % LANES;
  const int n = b.n_atoms;
  bool oor = false;
  if (a < T.count) {
    const int i = T.first + a;
    const double4 pi = pos[i];
    const double gix = G[i], giy = G[n + i], giz = G[2 * n + i];
    const double fp = saved[n + i], fpp = saved[2 * n + i];
    const int nn = nneigh[i] & MD_NN_MASK;
    const int cnt = nn > l ? (nn - l + LANES - 1) / LANES : 0;
    const size_t stride = (size_t)npad * LANES;
    const int* nb = neigh + (size_t)i * LANES + l;
    auto disp2 = [&](double x, double y, double z, double d[3]) {
      return pair_disp2(pi, x, y, z, len, inv, d);
    };
    // first visit: w_ij = (G_i - G_j) . (r_j - r_i) / r_ij = -s_ij
    const double k_phi = 0.25 * g.r_inv_h, k_rho = 0.5 * g.r_inv_h * fp;
    double tau_w = 0.0, umin = 0.0, umax = 0.0;
    adj_visit<U>(
        nb, stride, cnt, i,
        [&](int j) {
          const double4 p = pos[j];
          return AdjRec1{p.x, p.y, p.z, G[j], G[n + j], G[2 * n + j]};
        },
        [&](const AdjRec1& q) {
          double d[3];
          const double r2 = disp2(q.x, q.y, q.z, d);
          if (!(r2 < rc2)) return;
          const double ir = rsqrt_nr(r2);
          const double u = (r2 * ir - g.r_lo) * g.r_inv_h;
          umin = fmin(umin, u);
          umax = fmax(umax, u);
          double tt;
          const int k = interval_u(u, g.nr, tt);
          const double w = fma(gix - q.gx, d[0], fma(giy - q.gy, d[1], (giz - q.gz) * d[2])) * ir;
          const double t2 = tt * tt, s = 1.0 - tt;
          const double gb[4] = {-(s * s), tt * fma(3.0, tt, -4.0), fma(-3.0, t2, fma(2.0, tt, 1.0)),
                                t2};
          const double A = w * k_phi, B = w * k_rho;
          double dr = 0.0;
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) {
            atomicAdd(&b_phi[k + q4], gb[q4] * A);
            atomicAdd(&b_rho[k + q4], gb[q4] * B);
            dr = fma(c_rho[k + q4], gb[q4], dr);
          }
          tau_w = fma(dr, w, tau_w);
        });
    oor = umin < 0.0 || umax > (double)g.nr;
    // tau_i = sum_j rho'(r_ij) s_ij
    const double tau = -0.5 * g.r_inv_h * md_group_sum<LANES>(tau_w);
    if (JAC) {
      if (l == 0) s_w[a] = -fpp * tau;
    } else {
      const double cf = -fpp * tau * (1.0 / 6.0);
      adj_visit<U>(
          nb, stride, cnt, i,
          [&](int j) {
            const double4 p = pos[j];
            return make_double3(p.x, p.y, p.z);
          },
          [&](const double3& q) {
            double d[3];
            const double r2 = disp2(q.x, q.y, q.z, d);
            if (!(r2 < rc2)) return;
            double tt, bb[4];
            const int k = interval_u((r2 * rsqrt_nr(r2) - g.r_lo) * g.r_inv_h, g.nr, tt);
            basis6(tt, bb);
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) atomicAdd(&b_rho[k + q4], cf * bb[q4]);
          });
    }
    if (l == 0) {
      double tt, bb[4], gg[4];
      const int k = interval(saved[i], g.e_lo, g.e_inv_h, g.ne, tt, oor);
      bspline_basis(tt, bb, gg);
#pragma unroll
      for (int q = 0; q < 4; ++q) atomicAdd(&b_emb[k + q], -gg[q] * g.e_inv_h * tau);
    }
  }
  if (__any(oor)) {
    if ((threadIdx.x & (MD_WAVE - 1)) == 0) md_flag(ctl, MD_FLAG_TABLE_RANGE);
  }
  if (JAC) {
    __syncthreads();
    // into copy 0 of this wave's rho bins: lane k owns bin k, after the wave's own adds
    double* rho0 = bins + (size_t)wid * g.copies * g.stride + g.n_phi;
    const int lane = threadIdx.x & (MD_WAVE - 1);
    for (int k = lane; k < g.n_rho; k += MD_WAVE) {
      double acc = 0.0;
      for (int a2 = wid; a2 < T.count; a2 += nw)
        acc = fma(s_w[a2], __builtin_nontemporal_load(jac + (size_t)(T.first + a2) * g.n_rho + k),
                  acc);
      rho0[k] += acc;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < g.n_bins; q += blockDim.x) {
    double s = 0.0;
    if (q < n_hot) {
      for (int c = 0; c < n_copy; ++c) s += bins[(size_t)c * g.stride + q];
    } else {
      for (int w = 0; w < nw; ++w) s += emb_bins[(size_t)w * g.n_emb + q - n_hot];
    }
    tile_bins[(size_t)q * b.n_tiles + t] = s;
  }
}

// grad[q] = sum over tiles of the tile partials tile_bins[q][tile] (bin-major, so one
// block reads one contiguous row): thread h adds tiles h, h + 256, ... in order and
// the block's threads are combined in a fixed tree.
__global__ __launch_bounds__(256) void k_adj_reduce(const double* tile_bins, int n_tiles,
                                                    int n_bins, double* grad) {
  __shared__ double sh[4];
  const int q = blockIdx.x;
  double v[1] = {0.0};
  for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) v[0] += tile_bins[(size_t)q * n_tiles + t];
  md_block_sum<1>(v, sh);
  if (threadIdx.x == 0) grad[q] = v[0];
}

// Density Jacobian of fixed positions: jac[i][k] = d rhobar_i / d c_rho_k =
// sum_j beta_k(r_ij) over i's pairs within r_c.  Each atom of the tile owns an LDS
// row; its lanes add 6 beta in list order, and the row is scaled by 1/6 on the way out.
template <int LANES, int U>
__global__ __launch_bounds__(64 * LANES) void k_density_jacobian(
    md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, AdjGeom g, double rc2, double* jac,
    md_ctl_dev* ctl) {
  extern __shared__ double rows[];  // [64][n_rho]
  for (int q = threadIdx.x; q < MD_TILE * g.n_rho; q += blockDim.x) rows[q] = 0.0;
  __syncthreads();
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;
  const md_tile T = b.tiles[t];
  const md_domain& Dm = b.domains[T.rep];
  const double len[3] = {Dm.len[0], Dm.len[1], Dm.len[2]};
  const double inv[3] = {Dm.periodic[0] ? Dm.inv_len[0] : 0.0,
                         Dm.periodic[1] ? Dm.inv_len[1] : 0.0,
                         Dm.periodic[2] ? Dm.inv_len[2] : 0.0};
  const int a = threadIdx.x / LANES, l = threadIdx.x % LANES;
  bool oor = false;
  if (a < T.count) {
    const int i = T.first + a;
    const double4 pi = pos[i];
    const int nn = nneigh[i] & MD_NN_MASK;
    const int cnt = nn > l ? (nn - l + LANES - 1) / LANES : 0;
    double* row = rows + (size_t)a * g.n_rho;
    double umin = 0.0, umax = 0.0;
    adj_visit<U>(
        neigh + (size_t)i * LANES + l, (size_t)npad * LANES, cnt, i,
        [&](int j) {
          const double4 p = pos[j];
          return make_double3(p.x, p.y, p.z);
        },
        [&](const double3& q) {
          double d[3];
          const double r2 = pair_disp2(pi, q.x, q.y, q.z, len, inv, d);
          if (!(r2 < rc2)) return;
          const double u = (r2 * rsqrt_nr(r2) - g.r_lo) * g.r_inv_h;
          umin = fmin(umin, u);
          umax = fmax(umax, u);
          double tt, bb[4];
          const int k = interval_u(u, g.nr, tt);
          basis6(tt, bb);
#pragma unroll
          for (int q4 = 0; q4 < 4; ++q4) atomicAdd(&row[k + q4], bb[q4]);
        });
    oor = umin < 0.0 || umax > (double)g.nr;
  }
  if (__any(oor)) {
    if ((threadIdx.x & (MD_WAVE - 1)) == 0) md_flag(ctl, MD_FLAG_TABLE_RANGE);
  }
  __syncthreads();
  double* out = jac + (size_t)T.first * g.n_rho;
  for (int q = threadIdx.x; q < T.count * g.n_rho; q += blockDim.x) out[q] = rows[q] * (1.0 / 6.0);
}

// Force-matching loss and its cotangent: thread h of the fixed grid takes atoms
// h, h + G, h + 2G, ... (G threads in all) in order; blocks are combined by
// k_loss_final in block order, so the sum depends on n alone.
constexpr int MD_LOSS_BLOCK = 256, MD_LOSS_MAX_BLOCKS = 1024;

static inline int loss_blocks(int n) {
  const int g = (n + MD_LOSS_BLOCK - 1) / MD_LOSS_BLOCK;
  return g < MD_LOSS_MAX_BLOCKS ? (g > 0 ? g : 1) : MD_LOSS_MAX_BLOCKS;
}

template <typename R>
__global__ __launch_bounds__(MD_LOSS_BLOCK) void k_loss_partial(int n, const R* __restrict__ F,
                                                                const double* __restrict__ Fr,
                                                                double two_over_n, double* G,
                                                                double* part) {
  __shared__ double sh[MD_LOSS_BLOCK / MD_WAVE];
  double v[1] = {0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double d = (double)F[(size_t)c * n + i] - Fr[(size_t)c * n + i];
      v[0] = fma(d, d, v[0]);
      if (G) G[(size_t)c * n + i] = two_over_n * d;
    }
  }
  md_block_sum<1>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(MD_LOSS_BLOCK) void k_loss_final(int nb, const double* part,
                                                              double inv_n, double* loss) {
  __shared__ double sh[MD_LOSS_BLOCK / MD_WAVE];
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) v[0] += part[b];
  md_block_sum<1>(v, sh);
  if (threadIdx.x == 0) *loss = v[0] * inv_n;
}

bool adj_ok(const md_eam* p) {
  if (!p || !p->phi.coef || !p->rho.coef || !p->emb.coef) return false;
  if (p->phi.ncoef < 6 || p->rho.ncoef < 6 || p->emb.ncoef < 6) return false;
  if (p->phi.ncoef != p->rho.ncoef || p->phi.x_lo != p->rho.x_lo || p->phi.h != p->rho.h)
    return false;
  if (!(p->rho.h > 0.0) || !(p->emb.h > 0.0)) return false;
  return p->phi.ncoef + p->rho.ncoef + p->emb.ncoef <= MD_ADJ_MAX_BINS;
}

}  // namespace

extern "C" size_t md_backward_workspace_bytes(const md_batch* b, const md_eam* p) {
  if (!b || !adj_ok(p)) return 0;
  const size_t nb = (size_t)(p->phi.ncoef + p->rho.ncoef + p->emb.ncoef);
  return md_align256(8 * nb * (size_t)(b->n_tiles > 0 ? b->n_tiles : 1));
}

namespace {

AdjGeom adj_geom(const md_eam* p) {
  AdjGeom g;
  g.c_rho = p->rho.coef;
  g.r_lo = p->rho.x_lo;
  g.r_inv_h = 1.0 / p->rho.h;
  g.e_lo = p->emb.x_lo;
  g.e_inv_h = 1.0 / p->emb.h;
  g.nr = p->rho.ncoef - 3;
  g.ne = p->emb.ncoef - 3;
  g.n_phi = p->phi.ncoef;
  g.n_rho = p->rho.ncoef;
  g.n_emb = p->emb.ncoef;
  g.n_bins = g.n_phi + g.n_rho + g.n_emb;
  g.copies = 1;
  g.stride = g.n_phi + g.n_rho;
  return g;
}

bool lanes_ok(const md_nlist* nl) {
  const int L = nl->lanes;
  return (L == 1 || L == 2 || L == 4 || L == 8 || L == 16) && nl->max_neigh % L == 0;
}

int backward(const md_batch* b, const md_eam* p, md_precision prec, const double* pos,
             const md_nlist* nl, const double* saved, const double* jac,
             const double* grad_force, double* grad_coef, void* ws, void* ctl, void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if (!adj_ok(p) || !pos || !nl || !nl->neigh || !nl->nneigh || !saved || !grad_force ||
      !grad_coef || !ws || !ctl)
    return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (!lanes_ok(nl)) return MD_ERR_ARG;
  const int L = nl->lanes;
  AdjGeom g = adj_geom(p);
  hipStream_t st = (hipStream_t)stream;
  double* tile_bins = (double*)ws;
  const double rc2 = p->r_cut * p->r_cut;
  const int npad = md_npad(b->n_atoms);
  if (b->n_tiles > 0) {
    const dim3 grid(md_grid_blocks(b->n_tiles)), block(64 * L);
    const int nw = 64 * L / MD_WAVE, n_hot = g.n_phi + g.n_rho;
    g.stride = n_hot + (36 - n_hot % 32) % 32;  // copies start 8 banks apart
    const size_t extra = jac ? MD_TILE : 0;
    auto lds_of = [&](int c) {
      return ((size_t)nw * ((size_t)c * g.stride + g.n_emb) + g.n_rho + extra) * sizeof(double);
    };
    g.copies = jac ? MD_ADJ_COPIES_JAC : MD_ADJ_COPIES;
    while (g.copies > 1 && lds_of(g.copies) > MD_ADJ_LDS) g.copies >>= 1;
    const size_t lds = lds_of(g.copies);
    if (lds > 65536) return MD_ERR_ARG;  // fewer lanes per atom, or fewer coefficients
#define MD_ADJ_LAUNCH(LN, J)                                                                   \
  MD_LAUNCH_TIMED(MD_KERNEL_EAM_ADJOINT, (k_eam_adjoint<LN, MD_ADJ_U, J>), grid, block, lds,    \
                  st, *b, (const double4*)pos, nl->neigh, nl->nneigh, npad, saved, jac,         \
                  grad_force, g, rc2, tile_bins, (md_ctl_dev*)ctl)
#define MD_ADJ_LAUNCH_L(J)                \
  switch (L) {                            \
    case 1: MD_ADJ_LAUNCH(1, J); break;   \
    case 2: MD_ADJ_LAUNCH(2, J); break;   \
    case 4: MD_ADJ_LAUNCH(4, J); break;   \
    case 8: MD_ADJ_LAUNCH(8, J); break;   \
    default: MD_ADJ_LAUNCH(16, J); break; \
  }
    if (jac) {
      MD_ADJ_LAUNCH_L(true);
    } else {
      MD_ADJ_LAUNCH_L(false);
    }
#undef MD_ADJ_LAUNCH_L
#undef MD_ADJ_LAUNCH
    MD_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_adj_reduce, dim3(g.n_bins), dim3(256), 0, st, tile_bins, b->n_tiles,
                     g.n_bins, grad_coef);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

bool jac_ok(const md_eam* p) {
  return p && p->rho.ncoef >= 6 && p->rho.ncoef <= MD_JAC_MAX_COEF && p->rho.h > 0.0 &&
         p->r_cut > 0.0;
}

}  // namespace

extern "C" int md_eam_backward(const md_batch* b, const md_eam* p, md_precision prec,
                               const double* pos, const md_nlist* nl, const double* saved,
                               const double* grad_force, double* grad_coef, void* ws, void* ctl,
                               void* stream) {
  return backward(b, p, prec, pos, nl, saved, nullptr, grad_force, grad_coef, ws, ctl, stream);
}

extern "C" int md_eam_backward_jac(const md_batch* b, const md_eam* p, md_precision prec,
                                   const double* pos, const md_nlist* nl, const double* saved,
                                   const double* jac, const double* grad_force,
                                   double* grad_coef, void* ws, void* ctl, void* stream) {
  if (!jac) return MD_ERR_ARG;
  return backward(b, p, prec, pos, nl, saved, jac, grad_force, grad_coef, ws, ctl, stream);
}

extern "C" size_t md_density_jacobian_bytes(const md_batch* b, const md_eam* p) {
  if (!b || b->n_atoms < 0 || !jac_ok(p)) return 0;
  return md_align256(sizeof(double) * (size_t)b->n_atoms * p->rho.ncoef);
}

extern "C" int md_eam_density_jacobian(const md_batch* b, const md_eam* p, const double* pos,
                                       const md_nlist* nl, double* jac, void* ctl,
                                       void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if (!jac_ok(p) || !pos || !nl || !nl->neigh || !nl->nneigh || !jac || !ctl) return MD_ERR_ARG;
  if (!lanes_ok(nl)) return MD_ERR_ARG;
  if (b->n_tiles == 0) return MD_OK;
  const int L = nl->lanes;
  const AdjGeom g = adj_geom(p);
  const dim3 grid(md_grid_blocks(b->n_tiles)), block(64 * L);
  const size_t lds = (size_t)MD_TILE * g.n_rho * sizeof(double);
  hipStream_t st = (hipStream_t)stream;
  const double rc2 = p->r_cut * p->r_cut;
  const int npad = md_npad(b->n_atoms);
#define MD_JAC_LAUNCH(LN)                                                                    \
  hipLaunchKernelGGL((k_density_jacobian<LN, MD_ADJ_U>), grid, block, lds, st, *b,           \
                     (const double4*)pos, nl->neigh, nl->nneigh, npad, g, rc2, jac,         \
                     (md_ctl_dev*)ctl)
  switch (L) {
    case 1: MD_JAC_LAUNCH(1); break;
    case 2: MD_JAC_LAUNCH(2); break;
    case 4: MD_JAC_LAUNCH(4); break;
    case 8: MD_JAC_LAUNCH(8); break;
    default: MD_JAC_LAUNCH(16); break;
  }
#undef MD_JAC_LAUNCH
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" size_t md_force_loss_workspace_bytes(int n_atoms) {
  return n_atoms < 0 ? 0 : md_align256(sizeof(double) * (size_t)loss_blocks(n_atoms));
}

extern "C" int md_force_loss(int n_atoms, md_precision prec, const void* force, const double* f_ref,
                             double* loss, double* grad_force, void* ws, void* stream) {
  if (n_atoms < 0 || !loss || !ws) return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (n_atoms > 0 && (!force || !f_ref)) return MD_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)ws;
  const int nb = loss_blocks(n_atoms);
  if (n_atoms > 0) {
    const double two_over_n = 2.0 / n_atoms;
    if (prec == MD_FP64)
      hipLaunchKernelGGL(k_loss_partial<double>, dim3(nb), dim3(MD_LOSS_BLOCK), 0, st, n_atoms,
                         (const double*)force, f_ref, two_over_n, grad_force, part);
    else
      hipLaunchKernelGGL(k_loss_partial<float>, dim3(nb), dim3(MD_LOSS_BLOCK), 0, st, n_atoms,
                         (const float*)force, f_ref, two_over_n, grad_force, part);
    MD_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(MD_LOSS_BLOCK), 0, st, n_atoms > 0 ? nb : 0,
                     part, n_atoms > 0 ? 1.0 / n_atoms : 0.0, loss);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
