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
// tau_i).  Each wavefront accumulates into its own LDS bins; a block adds its
// wavefronts' bins in wave order into per-tile partials, and a second kernel
// adds the tile partials in tile order.  All sums are FP64.
#include <math.h>

#include "md_internal.h"

namespace {

#define MD_ADJ_MAX_BINS 1024

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
};

template <int LANES>
__global__ __launch_bounds__(64 * LANES) void k_eam_adjoint(
    md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, const double* __restrict__ saved,
    const double* __restrict__ G, AdjGeom g, double rc2, double* tile_bins, md_ctl_dev* ctl) {
  extern __shared__ double bins[];  // [waves][n_bins]
  const int nw = blockDim.x / MD_WAVE, wid = threadIdx.x / MD_WAVE;
  for (int q = threadIdx.x; q < nw * g.n_bins; q += blockDim.x) bins[q] = 0.0;
  __syncthreads();
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;
  double* wb = bins + (size_t)wid * g.n_bins;
  double* b_phi = wb;
  double* b_rho = wb + g.n_phi;
  double* b_emb = wb + g.n_phi + g.n_rho;
  const md_tile T = b.tiles[t];
  const md_domain& Dm = b.domains[T.rep];
  const int per[3] = {Dm.periodic[0], Dm.periodic[1], Dm.periodic[2]};
  const double len[3] = {Dm.len[0], Dm.len[1], Dm.len[2]};
  const double inv[3] = {Dm.inv_len[0], Dm.inv_len[1], Dm.inv_len[2]};
  const int a = threadIdx.x / LANES, l = threadIdx.x % LANES;
  const int n = b.n_atoms;
  bool oor = false;
  if (a < T.count) {
    const int i = T.first + a;
    const double4 pi = pos[i];
    const double gix = G[i], giy = G[n + i], giz = G[2 * n + i];
    const double fp = saved[n + i], fpp = saved[2 * n + i];
    const int nn = nneigh[i] & MD_NN_MASK;
    const size_t stride = (size_t)npad * LANES;
    double tau = 0.0;
    const int* nb = neigh + (size_t)i * LANES + l;
    for (int m = l; m < nn; m += LANES, nb += stride) {
      const int j = *nb;
      const double4 pj = pos[j];
      double d[3] = {pj.x - pi.x, pj.y - pi.y, pj.z - pi.z};
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (per[q]) d[q] -= len[q] * rint(d[q] * inv[q]);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (!(r2 < rc2)) continue;
      const double r = sqrt(r2), ir = 1.0 / r;
      // u_ij = (r_i - r_j) / r = -d / r
      const double s = -((gix - G[j]) * d[0] + (giy - G[n + j]) * d[1] + (giz - G[2 * n + j]) * d[2]) * ir;
      double tt, bb[4], gg[4];
      const int k = interval(r, g.r_lo, g.r_inv_h, g.nr, tt, oor);
      bspline_basis(tt, bb, gg);
      double drho = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double gq = gg[q] * g.r_inv_h;
        drho += g.c_rho[k + q] * gq;
        atomicAdd(&b_phi[k + q], -0.5 * gq * s);
        atomicAdd(&b_rho[k + q], -fp * gq * s);
      }
      tau += drho * s;
    }
    tau = md_group_sum<LANES>(tau);
    nb = neigh + (size_t)i * LANES + l;
    const double cf = -fpp * tau;
    for (int m = l; m < nn; m += LANES, nb += stride) {
      const int j = *nb;
      const double4 pj = pos[j];
      double d[3] = {pj.x - pi.x, pj.y - pi.y, pj.z - pi.z};
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (per[q]) d[q] -= len[q] * rint(d[q] * inv[q]);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (!(r2 < rc2)) continue;
      double tt, bb[4], gg[4];
      const int k = interval(sqrt(r2), g.r_lo, g.r_inv_h, g.nr, tt, oor);
      bspline_basis(tt, bb, gg);
#pragma unroll
      for (int q = 0; q < 4; ++q) atomicAdd(&b_rho[k + q], cf * bb[q]);
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
  __syncthreads();
  double* out = tile_bins + (size_t)t * g.n_bins;
  for (int q = threadIdx.x; q < g.n_bins; q += blockDim.x) {
    double s = bins[q];
    for (int w = 1; w < nw; ++w) s += bins[(size_t)w * g.n_bins + q];
    out[q] = s;
  }
}

// grad[q] = sum over tiles of tile_bins[tile][q], in tile order (one block per bin).
__global__ __launch_bounds__(256) void k_adj_reduce(const double* tile_bins, int n_tiles,
                                                    int n_bins, double* grad) {
  __shared__ double sh[4];
  const int q = blockIdx.x;
  double v[1] = {0.0};
  for (int t = threadIdx.x; t < n_tiles; t += blockDim.x) v[0] += tile_bins[(size_t)t * n_bins + q];
  md_block_sum<1>(v, sh);
  if (threadIdx.x == 0) grad[q] = v[0];
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

extern "C" int md_eam_backward(const md_batch* b, const md_eam* p, md_precision prec,
                               const double* pos, const md_nlist* nl, const double* saved,
                               const double* grad_force, double* grad_coef, void* ws, void* ctl,
                               void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if (!adj_ok(p) || !pos || !nl || !nl->neigh || !nl->nneigh || !saved || !grad_force ||
      !grad_coef || !ws || !ctl)
    return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  const int L = nl->lanes;
  if ((L != 1 && L != 2 && L != 4 && L != 8 && L != 16) || nl->max_neigh % L) return MD_ERR_ARG;
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
  hipStream_t st = (hipStream_t)stream;
  double* tile_bins = (double*)ws;
  const double rc2 = p->r_cut * p->r_cut;
  const int npad = md_npad(b->n_atoms);
  if (b->n_tiles > 0) {
    const dim3 grid(md_grid_blocks(b->n_tiles)), block(64 * L);
    const size_t lds = (size_t)(64 * L / MD_WAVE) * g.n_bins * sizeof(double);
    if (lds > 65536) return MD_ERR_ARG;  // fewer lanes per atom, or fewer coefficients
#define MD_ADJ_LAUNCH(LN)                                                                      \
  MD_LAUNCH_TIMED(MD_KERNEL_EAM_ADJOINT, k_eam_adjoint<LN>, grid, block, lds, st, *b,          \
                  (const double4*)pos, nl->neigh, nl->nneigh, npad, saved, grad_force, g, rc2, \
                  tile_bins, (md_ctl_dev*)ctl)
    switch (L) {
      case 1: MD_ADJ_LAUNCH(1); break;
      case 2: MD_ADJ_LAUNCH(2); break;
      case 4: MD_ADJ_LAUNCH(4); break;
      case 8: MD_ADJ_LAUNCH(8); break;
      default: MD_ADJ_LAUNCH(16); break;
    }
#undef MD_ADJ_LAUNCH
    MD_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_adj_reduce, dim3(g.n_bins), dim3(256), 0, st, tile_bins, b->n_tiles,
                     g.n_bins, grad_coef);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
