// Analysis path (Appendix): per-atom potential energy and pair virial in FP64,
// and slab profiles of the flow and thermodynamic fields.
#include <math.h>

#include "md_internal.h"

namespace {

constexpr double PROF_SCALE = 4294967296.0;  // 2^32 fixed-point units per unit

// Uniform cubic B-spline s(x) = sum_m c[i+m] b_m(t), u = (x - x_lo)/h, i = floor(u)
// clamped to the K - 1 intervals, t = u - i; value and first derivative.
struct Spl {
  const double* c;
  int K;  // breakpoints (ncoef - 2)
  double x_lo, h;
};

__device__ __forceinline__ Spl spl(const md_spline& s) { return Spl{s.coef, s.ncoef - 2, s.x_lo, s.h}; }

__device__ __forceinline__ double spl_eval(const Spl& s, double x, double& d1, bool& oor) {
  const double u = (x - s.x_lo) / s.h;
  if (!(u >= 0.0 && u <= (double)(s.K - 1))) oor = true;
  double fu = floor(u);
  if (!(fu >= 0.0)) fu = 0.0;
  if (fu > (double)(s.K - 2)) fu = (double)(s.K - 2);
  const int i = (int)fu;
  const double t = u - fu, w = 1.0 - t, t2 = t * t, t3 = t2 * t;
  const double c0 = s.c[i], c1 = s.c[i + 1], c2 = s.c[i + 2], c3 = s.c[i + 3];
  const double v = (c0 * w * w * w + c1 * (3.0 * t3 - 6.0 * t2 + 4.0) +
                    c2 * (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) + c3 * t3) / 6.0;
  d1 = (-c0 * w * w + c1 * (3.0 * t2 - 4.0 * t) + c2 * (-3.0 * t2 + 2.0 * t + 1.0) + c3 * t2) /
       (2.0 * s.h);
  return v;
}

// r_ij = x_i - x_j with the minimum image on periodic axes.
__device__ __forceinline__ void min_image(const md_domain& D, const double4& pi, const double4& pj,
                                          double (&d)[3]) {
  d[0] = pi.x - pj.x;
  d[1] = pi.y - pj.y;
  d[2] = pi.z - pj.z;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (D.periodic[a]) d[a] -= D.len[a] * rint(d[a] * D.inv_len[a]);
}

// Atom i of the per-atom grid-stride loop (256-thread blocks of 4 tiles); the
// body gets (i, tile).
template <typename Body>
__device__ __forceinline__ void for_atoms(const md_batch& b, Body body) {
  const int nlb = (b.n_tiles + 3) / 4;
  const int lane = threadIdx.x & (MD_WAVE - 1);
  for (int k = 0;; ++k) {
    const int lb = md_remap_stride(nlb, k);
    if (lb >= nlb) break;
    const int tile = lb * 4 + (int)(threadIdx.x / MD_WAVE);
    if (tile >= b.n_tiles) continue;
    const md_tile T = b.tiles[tile];
    if (lane >= T.count) continue;
    body(T.first + lane, T);
  }
}

__device__ __forceinline__ size_t list_entry(int i, int m, int lanes, size_t npad) {
  return ((size_t)(m / lanes) * npad + (size_t)i) * lanes + (size_t)(m % lanes);
}

// EAM, first pass: rhobar_i, F(rhobar_i), F'(rhobar_i), e_i = F + 1/2 sum_j phi(r_ij).
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_obs_eam_rho(md_batch b, md_eam p,
                                                               const double4* pos, md_nlist nl,
                                                               size_t npad, double* e_atom,
                                                               double* rho_fp, md_ctl_dev* ctl) {
  const Spl sphi = spl(p.phi), srho = spl(p.rho), semb = spl(p.emb);
  const double rc2 = p.r_cut * p.r_cut;
  bool oor = false;
  for_atoms(b, [&](int i, const md_tile& T) {
    const md_domain& D = b.domains[T.rep];
    const double4 pi = pos[i];
    const int nn = nl.nneigh[i] & MD_NN_MASK;
    double rho = 0.0, phi = 0.0, d1;
    for (int m = 0; m < nn; ++m) {
      const int j = nl.neigh[list_entry(i, m, nl.lanes, npad)];
      double d[3];
      min_image(D, pi, pos[j], d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 < rc2) {
        const double r = sqrt(r2);
        rho += spl_eval(srho, r, d1, oor);
        phi += spl_eval(sphi, r, d1, oor);
      }
    }
    double fp;
    const double F = spl_eval(semb, rho, fp, oor);
    e_atom[i] = F + 0.5 * phi;
    if (rho_fp) {
      rho_fp[i] = rho;
      rho_fp[b.n_atoms + i] = fp;
    }
  });
  if (__any(oor) && (threadIdx.x & (MD_WAVE - 1)) == 0) md_flag(ctl, MD_FLAG_TABLE_RANGE);
}

// EAM, second pass: w_i = 1/2 sum_j r_ij (x) f_ij with
// f_ij = -[phi'(r) + (F'_i + F'_j) rho'(r)] r_ij / r (F' from the first pass).
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_obs_eam_w(md_batch b, md_eam p,
                                                             const double4* pos, md_nlist nl,
                                                             size_t npad, const double* fp,
                                                             double* w_atom) {
  const Spl sphi = spl(p.phi), srho = spl(p.rho);
  const double rc2 = p.r_cut * p.r_cut;
  const int n = b.n_atoms;
  bool oor = false;
  for_atoms(b, [&](int i, const md_tile& T) {
    const md_domain& D = b.domains[T.rep];
    const double4 pi = pos[i];
    const double fpi = fp[i];
    const int nn = nl.nneigh[i] & MD_NN_MASK;
    double w[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < nn; ++m) {
      const int j = nl.neigh[list_entry(i, m, nl.lanes, npad)];
      double d[3];
      min_image(D, pi, pos[j], d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 < rc2) {
        const double r = sqrt(r2);
        double dphi, drho;
        spl_eval(sphi, r, dphi, oor);
        spl_eval(srho, r, drho, oor);
        const double s = -(dphi + (fpi + fp[j]) * drho) / r;  // f_ij = s r_ij
        w[0] += 0.5 * d[0] * s * d[0];
        w[1] += 0.5 * d[1] * s * d[1];
        w[2] += 0.5 * d[2] * s * d[2];
        w[3] += 0.5 * d[0] * s * d[1];
        w[4] += 0.5 * d[0] * s * d[2];
        w[5] += 0.5 * d[1] * s * d[2];
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) w_atom[(size_t)k * n + i] = w[k];
  });
}

// Lennard-Jones: e_i = 1/2 sum_j U(r_ij) (shifted), w_i = 1/2 sum_j r_ij (x) f_ij with
// f_ij = 24 eps [2 (s/r)^12 - (s/r)^6] r_ij / r^2.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_obs_lj(md_batch b, md_lj p, double ucut,
                                                          const double4* pos, md_nlist nl,
                                                          size_t npad, double* e_atom,
                                                          double* w_atom) {
  const double rc2 = p.r_cut * p.r_cut, sig2 = p.sigma * p.sigma;
  const int n = b.n_atoms;
  for_atoms(b, [&](int i, const md_tile& T) {
    const md_domain& D = b.domains[T.rep];
    const double4 pi = pos[i];
    const int nn = nl.nneigh[i] & MD_NN_MASK;
    double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < nn; ++m) {
      const int j = nl.neigh[list_entry(i, m, nl.lanes, npad)];
      double d[3];
      min_image(D, pi, pos[j], d);
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 < rc2) {
        const double sr2 = sig2 / r2, sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
        e += 0.5 * (4.0 * p.eps * (sr12 - sr6) - ucut);
        const double s = 24.0 * p.eps * (2.0 * sr12 - sr6) / r2;
        w[0] += 0.5 * d[0] * s * d[0];
        w[1] += 0.5 * d[1] * s * d[1];
        w[2] += 0.5 * d[2] * s * d[2];
        w[3] += 0.5 * d[0] * s * d[1];
        w[4] += 0.5 * d[0] * s * d[2];
        w[5] += 0.5 * d[1] * s * d[2];
      }
    }
    e_atom[i] = e;
#pragma unroll
    for (int k = 0; k < 6; ++k) w_atom[(size_t)k * n + i] = w[k];
  });
}

// ---------------------------------------------------------------------------
// Slab profiles.  Accumulators per bin (fixed point, PROF_SCALE units):
//   0 N, 1-3 sum v, 4 sum e, 5-10 sum w, 11-16 sum m dv (x) dv (eV), dv = v - u_l.
// ---------------------------------------------------------------------------
constexpr int NACC = 17;

struct ProfGeom {
  int axis, n_bins;
  double lo, width;
};

__device__ __forceinline__ int bin_of(const md_domain& D, const ProfGeom& G, const double4& p) {
  const int a = G.axis;
  double x = a == 0 ? p.x : (a == 1 ? p.y : p.z);
  if (D.periodic[a]) {
    x = x - D.len[a] * floor((x - D.lo[a]) / D.len[a]);
    if (x >= D.lo[a] + D.len[a]) x = D.lo[a];
  }
  const double q = floor((x - G.lo) / G.width);
  return (q >= 0.0 && q < (double)G.n_bins) ? (int)q : -1;
}

// Add v[0..NQ) of every lane into acc[bin * NACC + base + q]: one wave-wide sum and
// one integer atomic per distinct bin of the wave (atoms in cell order share few bins).
template <int NQ>
__device__ __forceinline__ void wave_bin_add(int bin, const double (&v)[NQ], long long* acc,
                                             int base) {
  unsigned long long left = __ballot(bin >= 0);
  const int lane = threadIdx.x & (MD_WAVE - 1);
  while (left) {
    const int leader = __ffsll((long long)left) - 1;
    const int lb = __shfl(bin, leader, MD_WAVE);
    const bool mine = bin == lb;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double s = md_wave_sum(mine ? v[q] : 0.0);
      if (lane == 0)
        atomicAdd((unsigned long long*)&acc[(size_t)lb * NACC + base + q],
                  (unsigned long long)(long long)rint(s * PROF_SCALE));
    }
    left &= ~__ballot(mine);
  }
}

__global__ void k_prof_zero(long long* acc, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    acc[k] = 0;
}

// Every lane of a wave takes part in the wave-wide sums, so the loops run over whole
// tiles (lanes past a tile's end contribute no bin).
template <typename Body>
__device__ __forceinline__ void for_tiles(const md_batch& b, Body body) {
  const int nlb = (b.n_tiles + 3) / 4;
  const int lane = threadIdx.x & (MD_WAVE - 1);
  for (int k = 0;; ++k) {
    const int lb = md_remap_stride(nlb, k);
    if (lb >= nlb) break;
    const int tile = lb * 4 + (int)(threadIdx.x / MD_WAVE);
    if (tile >= b.n_tiles) continue;  // uniform across the wave
    const md_tile T = b.tiles[tile];
    body(lane < T.count ? T.first + lane : -1, T);
  }
}

__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_prof_pass1(md_batch b, ProfGeom G,
                                                              const double4* pos,
                                                              const double* vel,
                                                              const double* e_atom,
                                                              const double* w_atom,
                                                              long long* acc) {
  const int n = b.n_atoms;
  for_tiles(b, [&](int i, const md_tile& T) {
    int bin = -1;
    double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i >= 0) {
      bin = bin_of(b.domains[T.rep], G, pos[i]);
      v[0] = 1.0;
      v[1] = vel[i];
      v[2] = vel[n + i];
      v[3] = vel[2 * n + i];
      if (e_atom) v[4] = e_atom[i];
      if (w_atom)
#pragma unroll
        for (int k = 0; k < 6; ++k) v[5 + k] = w_atom[(size_t)k * n + i];
    }
    wave_bin_add<11>(bin, v, acc, 0);
  });
}

__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_prof_pass2(md_batch b, ProfGeom G,
                                                              const double4* pos,
                                                              const double* vel, double mass,
                                                              long long* acc) {
  const int n = b.n_atoms;
  const double m_e = mass / MD_ACCEL;  // u (angstrom/ps)^2 -> eV
  for_tiles(b, [&](int i, const md_tile& T) {
    int bin = -1;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i >= 0) {
      bin = bin_of(b.domains[T.rep], G, pos[i]);
      if (bin >= 0) {
        const long long* a = acc + (size_t)bin * NACC;
        const double cnt = (double)a[0] / PROF_SCALE;
        const double dv[3] = {vel[i] - (double)a[1] / PROF_SCALE / cnt,
                              vel[n + i] - (double)a[2] / PROF_SCALE / cnt,
                              vel[2 * n + i] - (double)a[3] / PROF_SCALE / cnt};
        v[0] = m_e * dv[0] * dv[0];
        v[1] = m_e * dv[1] * dv[1];
        v[2] = m_e * dv[2] * dv[2];
        v[3] = m_e * dv[0] * dv[1];
        v[4] = m_e * dv[0] * dv[2];
        v[5] = m_e * dv[1] * dv[2];
      }
    }
    wave_bin_add<6>(bin, v, acc, 11);
  });
}

// out[bin][MD_PROF_LEN]: N, M, u[3], T^x, T^y, T^z, T, P^{xx yy zz xy xz yz}, P,
// E_pot / M, E_int / M.
__global__ void k_prof_final(md_batch b, int axis, double width, int n_bins,
                             const long long* acc, double mass, double* out) {
  const double kB = 8.617333262e-5;
  const md_domain& D = b.domains[0];
  double volume = width;  // bin width times the box cross-section
  for (int a = 0; a < 3; ++a)
    if (a != axis) volume *= D.len[a];
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_bins; l += gridDim.x * blockDim.x) {
    const long long* a = acc + (size_t)l * NACC;
    double* o = out + (size_t)l * MD_PROF_LEN;
    const double N = (double)a[0] / PROF_SCALE;
    if (!(N > 0.0)) {
      for (int k = 0; k < MD_PROF_LEN; ++k) o[k] = 0.0;
      continue;
    }
    const double M = N * mass;
    double K[6], W[6];
    for (int k = 0; k < 6; ++k) {
      K[k] = (double)a[11 + k] / PROF_SCALE;
      W[k] = (double)a[5 + k] / PROF_SCALE;
    }
    o[0] = N;
    o[1] = M;
    for (int k = 0; k < 3; ++k) o[2 + k] = (double)a[1 + k] / PROF_SCALE / N;
    for (int k = 0; k < 3; ++k) o[5 + k] = K[k] / (kB * N);
    o[8] = (o[5] + o[6] + o[7]) / 3.0;
    for (int k = 0; k < 6; ++k) o[9 + k] = (K[k] + W[k]) / volume;
    o[15] = (o[9] + o[10] + o[11]) / 3.0;
    const double epot = (double)a[4] / PROF_SCALE;
    o[16] = epot / M;
    o[17] = (epot + 0.5 * (K[0] + K[1] + K[2])) / M;
  }
}

bool spline_ok(const md_spline& s) { return s.coef && s.ncoef >= 6 && s.h > 0.0; }

}  // namespace

extern "C" int md_atom_observables(const md_batch* b, const md_eam* eam, const md_lj* lj,
                                   const double* pos, const md_nlist* nl, double* e_atom,
                                   double* w_atom, double* rho_fp, void* ctl, void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if ((eam == nullptr) == (lj == nullptr)) return MD_ERR_ARG;
  if (!pos || !nl || !nl->neigh || !nl->nneigh || !e_atom || !w_atom || !ctl) return MD_ERR_ARG;
  if (nl->lanes < 1 || nl->lanes > MD_MAX_LANES || nl->max_neigh < nl->lanes) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
  const size_t npad = (size_t)md_npad(b->n_atoms);
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  if (lj) {
    if (!(lj->sigma > 0.0) || !(lj->r_cut > 0.0)) return MD_ERR_ARG;
    const double sr6 = pow(lj->sigma / lj->r_cut, 6.0);
    const double ucut = 4.0 * lj->eps * (sr6 * sr6 - sr6);
    hipLaunchKernelGGL(k_obs_lj, grid, block, 0, st, *b, *lj, ucut, (const double4*)pos, *nl,
                       npad, e_atom, w_atom);
    MD_LAUNCH_CHECK();
    return MD_OK;
  }
  if (!spline_ok(eam->phi) || !spline_ok(eam->rho) || !spline_ok(eam->emb) || !rho_fp ||
      !(eam->r_cut > 0.0))
    return MD_ERR_ARG;
  hipLaunchKernelGGL(k_obs_eam_rho, grid, block, 0, st, *b, *eam, (const double4*)pos, *nl, npad,
                     e_atom, rho_fp, c);
  MD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_obs_eam_w, grid, block, 0, st, *b, *eam, (const double4*)pos, *nl, npad,
                     (const double*)(rho_fp + b->n_atoms), w_atom);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" size_t md_profile_workspace_bytes(int n_bins) {
  return n_bins > 0 ? md_align256((size_t)n_bins * NACC * sizeof(long long)) : 0;
}

extern "C" int md_profiles(const md_batch* b, int axis, double lo, double width, int n_bins,
                           const double* pos, const double* vel, double mass,
                           const double* e_atom, const double* w_atom, double* out, void* ws,
                           void* stream) {
  if (!md_batch_ok(b) || b->n_rep != 1) return MD_ERR_ARG;
  if (axis < 0 || axis > 2 || !(width > 0.0) || !isfinite(lo) || n_bins < 1 ||
      n_bins > MD_MAX_PROFILE_BINS || !(mass > 0.0))
    return MD_ERR_ARG;
  if (!pos || !vel || !out || !ws) return MD_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  long long* acc = (long long*)ws;
  const int n_acc = n_bins * NACC;
  hipLaunchKernelGGL(k_prof_zero, dim3((n_acc + 255) / 256), dim3(256), 0, st, acc, n_acc);
  MD_LAUNCH_CHECK();
  if (b->n_atoms > 0) {
    const ProfGeom G{axis, n_bins, lo, width};
    const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
    hipLaunchKernelGGL(k_prof_pass1, grid, block, 0, st, *b, G, (const double4*)pos, vel, e_atom,
                       w_atom, acc);
    MD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_prof_pass2, grid, block, 0, st, *b, G, (const double4*)pos, vel, mass,
                       acc);
    MD_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_prof_final, dim3((n_bins + 255) / 256), dim3(256), 0, st, *b, axis, width,
                     n_bins, acc, mass, out);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
