// Behler-Parrinello network potential (Sec. 2.1) in FP64: symmetry functions,
// the atomic network with its backward pass, and forces by the chain rule (eq. force).
//
// One wavefront per atom.  Its neighbours within r_cut are compacted into LDS; the
// radial functions take lanes over neighbours, the angular ones lanes over the unordered
// pairs j < k with R_jk < r_cut, compacted a wavefront at a time (the summand is
// symmetric in j and k, so each unordered pair stands for both ordered ones).  The G4
// set is a grid of distinct eta values (index u) and distinct (zeta, lambda) pairs
// (index v): per pair the
// lane evaluates exp(-eta_u s2) and (1 + lambda_v cos)^zeta_v once each and
// accumulates their products on the grid, so the cost per pair does not grow with
// the number of G4 functions that share them.
#include <math.h>

#include "md_internal.h"

namespace {

constexpr int NE = 8;  // distinct G4 eta values
constexpr int NZ = 8;  // distinct (zeta, lambda) pairs
constexpr int WPB = 4; // waves (atoms in flight) per block
constexpr double PI = 3.14159265358979323846;

struct BpnnDev {
  double rc, rc2, rs;
  int n2, n4, ng, h1, h2, n_eta, n_zl;
  double g2_eta[MD_BPNN_MAX_G];
  double eta_u[NE], zeta_v[NZ], lam_v[NZ];
  int izeta_v[NZ];  // zeta as an integer (>= 1) or 0 when not integral
  double pref[MD_BPNN_MAX_G];
  unsigned char u_of[MD_BPNN_MAX_G], v_of[MD_BPNN_MAX_G];
  const double* w;  // w01 [ng][h1], b1 [h1], w12 [h1][h2], b2 [h2], w23 [h2], b3
};

// Neighbours of one atom within r_cut, compacted in LDS.
struct Nb {
  double ax[MD_BPNN_MAX_NB], ay[MD_BPNN_MAX_NB], az[MD_BPNN_MAX_NB];
  double R[MD_BPNN_MAX_NB], iR[MD_BPNN_MAX_NB], fc[MD_BPNN_MAX_NB], dfc[MD_BPNN_MAX_NB];
  double gx[MD_BPNN_MAX_NB], gy[MD_BPNN_MAX_NB], gz[MD_BPNN_MAX_NB];
  int j[MD_BPNN_MAX_NB];
  double G[MD_BPNN_MAX_G];
  double h1[MD_BPNN_MAX_HIDDEN], h2[MD_BPNN_MAX_HIDDEN], d1[MD_BPNN_MAX_HIDDEN],
      d2[MD_BPNN_MAX_HIDDEN];
  double C[NE * NZ];
  unsigned short pq[2 * MD_WAVE];  // queued neighbour pairs j | k << 8 (for_pairs_in_cutoff)
  int nc;
};

__device__ __forceinline__ void cutoff(double R, double rc, double& fc, double& dfc) {
  if (R < rc) {
    double s, c;
    sincospi(R / rc, &s, &c);  // sin and cos of pi R / r_c (argument reduction is exact)
    fc = 0.5 * (c + 1.0);
    dfc = -0.5 * PI / rc * s;
  } else {
    fc = 0.0;
    dfc = 0.0;
  }
}

// x^n for an integer n >= 0 by binary powering, or pow(x, y) when n = 0 marks a
// non-integral exponent.
__device__ __forceinline__ double powi(double x, int n, double y) {
  if (n <= 0) return n == 0 && y != 0.0 ? pow(x, y) : 1.0;
  double r = 1.0;
  while (n) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

// Stage atom i's neighbours within r_cut into LDS (lane-parallel, order of the list).
__device__ void gather_neighbours(const BpnnDev& P, const md_domain& D, const double4* pos,
                                  const md_nlist& nl, size_t npad, int i, Nb& s, bool& over) {
  const int lane = threadIdx.x & (MD_WAVE - 1);
  const int nn = nl.nneigh[i] & MD_NN_MASK;
  const double4 pi = pos[i];
  int base = 0;
  for (int m0 = 0; m0 < nn; m0 += MD_WAVE) {
    const int m = m0 + lane;
    bool keep = false;
    double a[3] = {0, 0, 0}, r2 = 0.0;
    int j = 0;
    if (m < nn) {
      j = nl.neigh[((size_t)(m / nl.lanes) * npad + (size_t)i) * nl.lanes + (m % nl.lanes)];
      const double4 pj = pos[j];
      a[0] = pj.x - pi.x;
      a[1] = pj.y - pi.y;
      a[2] = pj.z - pi.z;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (D.periodic[q]) a[q] -= D.len[q] * rint(a[q] * D.inv_len[q]);
      r2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
      keep = r2 < P.rc2;
    }
    const unsigned long long mask = __ballot(keep);
    const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
    if (keep && slot < MD_BPNN_MAX_NB) {
      const double R = sqrt(r2);
      double fc, dfc;
      cutoff(R, P.rc, fc, dfc);
      s.ax[slot] = a[0];
      s.ay[slot] = a[1];
      s.az[slot] = a[2];
      s.R[slot] = R;
      s.iR[slot] = 1.0 / R;  // divisions per pair become products
      s.fc[slot] = fc;
      s.dfc[slot] = dfc;
      s.gx[slot] = 0.0;
      s.gy[slot] = 0.0;
      s.gz[slot] = 0.0;
      s.j[slot] = j;
    }
    base += __popcll(mask);
  }
  if (base > MD_BPNN_MAX_NB) over = true;
  if (lane == 0) s.nc = base < MD_BPNN_MAX_NB ? base : MD_BPNN_MAX_NB;
  __builtin_amdgcn_wave_barrier();
}

// Geometry of the ordered pair (j, k) of neighbours of the centre atom.
struct Trip {
  double cos, C, fC, dfC, s2, f3;
};

__device__ __forceinline__ Trip triplet(const BpnnDev& P, const Nb& s, int j, int k) {
  Trip t;
  const double dx = s.ax[k] - s.ax[j], dy = s.ay[k] - s.ay[j], dz = s.az[k] - s.az[j];
  const double A = s.R[j], B = s.R[k];
  t.C = sqrt(dx * dx + dy * dy + dz * dz);
  cutoff(t.C, P.rc, t.fC, t.dfC);
  // |cos| <= 1 up to rounding; clamped so that a non-integral zeta never meets a
  // negative base
  t.cos = fmin(1.0, fmax(-1.0, (s.ax[j] * s.ax[k] + s.ay[j] * s.ay[k] + s.az[j] * s.az[k]) *
                                   (s.iR[j] * s.iR[k])));
  t.s2 = A * A + B * B + t.C * t.C;
  t.f3 = s.fc[j] * s.fc[k] * t.fC;
  return t;
}

// Unordered pair t (0 <= t < nc (nc - 1) / 2) -> (j, k), j < k, row-major over j:
// row j holds the nc - 1 - j pairs (j, j + 1 .. nc - 1) and starts at
// off(j) = j (2 nc - j - 1) / 2.
__device__ __forceinline__ void pair_of(int t, int nc, int& j, int& k) {
  const double b = 2.0 * nc - 1.0;
  int r = (int)floor(0.5 * (b - sqrt(b * b - 8.0 * (double)t)));
  r = r < 0 ? 0 : (r > nc - 2 ? nc - 2 : r);
  while (r > 0 && r * (2 * nc - r - 1) / 2 > t) --r;
  while (r < nc - 2 && (r + 1) * (2 * nc - r - 2) / 2 <= t) ++r;
  j = r;
  k = t - r * (2 * nc - r - 1) / 2 + r + 1;
}

// The centre atom's unordered neighbour pairs j < k with R_jk < r_cut, a wavefront at a
// time.  Lanes test 64 flat pair indices per trip and append the accepted pairs to an LDS
// queue; each full wavefront of queued pairs, and the remainder at the end, goes to
// body(j, k, active).  A pair beyond the cutoff adds nothing to G4 or to its derivatives
// (f_c(R_jk) = f_c'(R_jk) = 0), and about half the pairs of a neighbour sphere are such
// pairs: compacting them away keeps the lanes on pairs that contribute.
template <typename Body>
__device__ __forceinline__ void for_pairs_in_cutoff(const BpnnDev& P, Nb& s, int nc, Body body) {
  const int lane = threadIdx.x & (MD_WAVE - 1);
  const int npairs = nc * (nc - 1) / 2;
  int qn = 0;  // queued pairs (below 64 between trips)
  for (int t0 = 0; t0 < npairs; t0 += MD_WAVE) {
    const int t = t0 + lane;
    bool ok = false;
    int j = 0, k = 0;
    if (t < npairs) {
      pair_of(t, nc, j, k);
      const double dx = s.ax[k] - s.ax[j], dy = s.ay[k] - s.ay[j], dz = s.az[k] - s.az[j];
      ok = sqrt(dx * dx + dy * dy + dz * dz) < P.rc;  // the test cutoff() applies to R_jk
    }
    const unsigned long long m = __ballot(ok);
    if (ok) s.pq[qn + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned short)(j | (k << 8));
    qn += __popcll(m);
    __builtin_amdgcn_wave_barrier();
    if (qn >= MD_WAVE) {
      const unsigned e = s.pq[lane];
      const unsigned rest = lane < qn - MD_WAVE ? s.pq[MD_WAVE + lane] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (lane < qn - MD_WAVE) s.pq[lane] = (unsigned short)rest;
      qn -= MD_WAVE;
      __builtin_amdgcn_wave_barrier();
      body((int)(e & 255u), (int)(e >> 8), true);
    }
  }
  if (qn > 0) {
    const unsigned e = lane < qn ? s.pq[lane] : 0u;
    body((int)(e & 255u), (int)(e >> 8), lane < qn);
  }
  __builtin_amdgcn_wave_barrier();
}

// Pass 1: symmetry functions, E_i and dE_i/dG per atom.  NEU eta values are kept in the
// per-lane accumulator grid (NEU x NZ registers): 6 for sets with at most six distinct
// eta values (the common case, which leaves room for two wavefronts per SIMD), else NE.
template <int NEU>
__global__ __launch_bounds__(64 * WPB, 2) void k_bpnn_desc(md_batch b, BpnnDev P, const double4* pos,
                                                        md_nlist nl, size_t npad, double* dEdG,
                                                        double* e_buf, md_ctl_dev* ctl) {
  __shared__ Nb sh[WPB];
  md_step_bookkeeping(ctl);
  const int w = threadIdx.x / MD_WAVE, lane = threadIdx.x & (MD_WAVE - 1);
  Nb& s = sh[w];
  const md_tile T = b.tiles[blockIdx.x];
  const md_domain& D = b.domains[T.rep];
  bool over = false;
  for (int a = w; a < T.count; a += WPB) {
    const int i = T.first + a;
    gather_neighbours(P, D, pos, nl, npad, i, s, over);
    const int nc = s.nc;
    // radial functions: lanes over neighbours
    for (int mu = 0; mu < P.n2; ++mu) {
      double acc = 0.0;
      for (int m = lane; m < nc; m += MD_WAVE) {
        const double d = s.R[m] - P.rs;
        acc += exp(-P.g2_eta[mu] * d * d) * s.fc[m];
      }
      acc = md_wave_sum(acc);
      if (lane == 0) s.G[mu] = acc;
    }
    // angular functions: lanes over the unordered pairs within the cutoff
    double g[NEU][NZ];
#pragma unroll
    for (int u = 0; u < NEU; ++u)
#pragma unroll
      for (int v = 0; v < NZ; ++v) g[u][v] = 0.0;
    for_pairs_in_cutoff(P, s, nc, [&](int j, int k, bool active) {
      if (!active) return;
      const Trip t = triplet(P, s, j, k);
      if (t.f3 == 0.0) return;
      double X[NEU], Pw[NZ];
#pragma unroll
      for (int u = 0; u < NEU; ++u) X[u] = u < P.n_eta ? exp(-P.eta_u[u] * t.s2) * t.f3 : 0.0;
#pragma unroll
      for (int v = 0; v < NZ; ++v)
        Pw[v] = v < P.n_zl ? powi(1.0 + P.lam_v[v] * t.cos, P.izeta_v[v], P.zeta_v[v]) : 0.0;
#pragma unroll
      for (int u = 0; u < NEU; ++u)
#pragma unroll
        for (int v = 0; v < NZ; ++v) g[u][v] += X[u] * Pw[v];
    });
#pragma unroll
    for (int u = 0; u < NEU; ++u)
#pragma unroll
      for (int v = 0; v < NZ; ++v) g[u][v] = md_wave_sum(g[u][v]);
    if (lane < P.n4) {
      double val = 0.0;
#pragma unroll
      for (int u = 0; u < NEU; ++u)
#pragma unroll
        for (int v = 0; v < NZ; ++v)
          if (u == P.u_of[lane] && v == P.v_of[lane]) val = g[u][v];
      s.G[P.n2 + lane] = 2.0 * P.pref[lane] * val;  // both orders of each pair
    }
    __builtin_amdgcn_wave_barrier();
    // the atomic network and its backward pass
    const double* w01 = P.w;
    const double* b1 = w01 + (size_t)P.ng * P.h1;
    const double* w12 = b1 + P.h1;
    const double* b2 = w12 + (size_t)P.h1 * P.h2;
    const double* w23 = b2 + P.h2;
    const double b3 = w23[P.h2];
    if (lane < P.h1) {
      double x = b1[lane];
      for (int mu = 0; mu < P.ng; ++mu) x += s.G[mu] * w01[(size_t)mu * P.h1 + lane];
      s.h1[lane] = tanh(x);
    }
    __builtin_amdgcn_wave_barrier();
    double e_part = 0.0;
    if (lane < P.h2) {
      double x = b2[lane];
      for (int q = 0; q < P.h1; ++q) x += s.h1[q] * w12[(size_t)q * P.h2 + lane];
      const double h = tanh(x);
      s.h2[lane] = h;
      s.d2[lane] = w23[lane] * (1.0 - h * h);
      e_part = w23[lane] * h;
    }
    const double E = b3 + md_wave_sum(e_part);
    __builtin_amdgcn_wave_barrier();
    if (lane < P.h1) {
      double x = 0.0;
      for (int q = 0; q < P.h2; ++q) x += w12[(size_t)lane * P.h2 + q] * s.d2[q];
      const double h = s.h1[lane];
      s.d1[lane] = x * (1.0 - h * h);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < P.ng) {
      double x = 0.0;
      for (int q = 0; q < P.h1; ++q) x += w01[(size_t)lane * P.h1 + q] * s.d1[q];
      dEdG[(size_t)i * P.ng + lane] = x;
    }
    if (lane == 0) e_buf[i] = E;
    __builtin_amdgcn_wave_barrier();
  }
  if (__any(over) && lane == 0) md_flag(ctl, MD_FLAG_NEIGH_OVERFLOW);
}

// Add a block's sums v[0..7) (E, W[6]) into the record as fixed point.
__device__ __forceinline__ void block_record_add(double (&v)[7], double* red, long long* slot,
                                                 int rep) {
  const int w = threadIdx.x / MD_WAVE, lane = threadIdx.x & (MD_WAVE - 1);
#pragma unroll
  for (int q = 0; q < 7; ++q) v[q] = md_wave_sum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 7; ++q) red[w * 7 + q] = v[q];
  __syncthreads();
  if (threadIdx.x < 7) {
    double s = 0.0;
    for (int q = 0; q < WPB; ++q) s += red[q * 7 + threadIdx.x];
    atomicAdd((unsigned long long*)&slot[(size_t)rep * MD_EV_LEN + threadIdx.x],
              (unsigned long long)(long long)rint(s * MD_EV_SCALE));
  }
}

// Pass 2: forces.  g_m = dE_i/d a_m for every neighbour vector a_m = x_j - x_i;
// F_j -= g_m, F_i += sum_m g_m, W -= a_m (x) g_m.
__global__ __launch_bounds__(64 * WPB, 3) void k_bpnn_force(md_batch b, BpnnDev P,
                                                         const double4* pos, md_nlist nl,
                                                         size_t npad, const double* dEdG,
                                                         const double* e_buf, double* force,
                                                         long long* ev, int ev_cap,
                                                         md_ctl_dev* ctl) {
  __shared__ Nb sh[WPB];
  __shared__ double red[WPB * 7];
  const int w = threadIdx.x / MD_WAVE, lane = threadIdx.x & (MD_WAVE - 1);
  Nb& s = sh[w];
  const md_tile T = b.tiles[blockIdx.x];
  const md_domain& D = b.domains[T.rep];
  const int n = b.n_atoms;
  bool over = false;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // E, W xx yy zz xy xz yz
  for (int a = w; a < T.count; a += WPB) {
    const int i = T.first + a;
    gather_neighbours(P, D, pos, nl, npad, i, s, over);
    const int nc = s.nc;
    const double* c = dEdG + (size_t)i * P.ng;
    // grid weights of the angular terms
    for (int q = lane; q < NE * NZ; q += MD_WAVE) s.C[q] = 0.0;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0)
      for (int q = 0; q < P.n4; ++q)
        s.C[P.u_of[q] * NZ + P.v_of[q]] += 2.0 * c[P.n2 + q] * P.pref[q];  // both orders
    __builtin_amdgcn_wave_barrier();
    // radial terms: lanes over neighbours
    for (int m = lane; m < nc; m += MD_WAVE) {
      const double R = s.R[m], d = R - P.rs, fc = s.fc[m], dfc = s.dfc[m];
      double dR = 0.0;
      for (int mu = 0; mu < P.n2; ++mu) {
        const double eta = P.g2_eta[mu];
        dR += c[mu] * exp(-eta * d * d) * (dfc - 2.0 * eta * d * fc);
      }
      const double q = dR / R;
      s.gx[m] += q * s.ax[m];
      s.gy[m] += q * s.ay[m];
      s.gz[m] += q * s.az[m];
    }
    __builtin_amdgcn_wave_barrier();
    // angular terms: lanes over the unordered pairs j < k within the cutoff.  The pair
    // (j, k) adds g_a to neighbour j and g_b to k; the reversed order adds the same
    // vectors with the roles swapped, which the factor 2 in the grid weights C accounts
    // for.  Lanes of one step can share a neighbour, so the LDS sums take atomic adds.
    for_pairs_in_cutoff(P, s, nc, [&](int j, int k, bool active) {
      if (!active) return;
      const Trip t = triplet(P, s, j, k);
      double X[NE], Pw[NZ], Pw1[NZ];
#pragma unroll
      for (int u = 0; u < NE; ++u) X[u] = u < P.n_eta ? exp(-P.eta_u[u] * t.s2) : 0.0;
      const double cz = t.cos;
#pragma unroll
      for (int v = 0; v < NZ; ++v) {
        const double base = 1.0 + P.lam_v[v] * cz;
        const int iz = P.izeta_v[v];
        Pw1[v] = v < P.n_zl ? powi(base, iz > 0 ? iz - 1 : 0, P.zeta_v[v] - 1.0) : 0.0;
        Pw[v] = Pw1[v] * base;
      }
      double q1 = 0.0, qe = 0.0, qc = 0.0;
#pragma unroll
      for (int u = 0; u < NE; ++u)
#pragma unroll
        for (int v = 0; v < NZ; ++v) {
          const double cw = s.C[u * NZ + v] * X[u];
          q1 += cw * Pw[v];
          qe += cw * Pw[v] * P.eta_u[u];
          qc += cw * P.zeta_v[v] * P.lam_v[v] * Pw1[v];
        }
      const double A = s.R[j], B = s.R[k], Cd = t.C;
      const double fA = s.fc[j], dfA = s.dfc[j], fB = s.fc[k], dfB = s.dfc[k];
      const double s_cos = qc * t.f3;
      const double sA = q1 * dfA * fB * t.fC - 2.0 * A * qe * t.f3;
      const double sB = q1 * fA * dfB * t.fC - 2.0 * B * qe * t.f3;
      const double sC = q1 * fA * fB * t.dfC - 2.0 * Cd * qe * t.f3;
      const double aj[3] = {s.ax[j], s.ay[j], s.az[j]}, ak[3] = {s.ax[k], s.ay[k], s.az[k]};
      const double iA = s.iR[j], iB = s.iR[k], iC = 1.0 / Cd;
      const double iAB = iA * iB, cA = t.cos * (iA * iA), cB = t.cos * (iB * iB);
      const double rA = sA * iA, rB = sB * iB, rC = sC * iC;
      double ga[3], gb[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double d = ak[q] - aj[q];
        ga[q] = s_cos * (ak[q] * iAB - cA * aj[q]) + rA * aj[q] - rC * d;
        gb[q] = s_cos * (aj[q] * iAB - cB * ak[q]) + rB * ak[q] + rC * d;
      }
      atomicAdd(&s.gx[j], ga[0]);
      atomicAdd(&s.gy[j], ga[1]);
      atomicAdd(&s.gz[j], ga[2]);
      atomicAdd(&s.gx[k], gb[0]);
      atomicAdd(&s.gy[k], gb[1]);
      atomicAdd(&s.gz[k], gb[2]);
    });
    __builtin_amdgcn_wave_barrier();
    // scatter: F_j -= g, F_i += sum g, W -= a (x) g
    double fi[3] = {0, 0, 0}, wv[6] = {0, 0, 0, 0, 0, 0};
    for (int m = lane; m < nc; m += MD_WAVE) {
      const double g[3] = {s.gx[m], s.gy[m], s.gz[m]};
      const double av[3] = {s.ax[m], s.ay[m], s.az[m]};
      const int j = s.j[m];
      atomicAdd(&force[j], -g[0]);
      atomicAdd(&force[n + j], -g[1]);
      atomicAdd(&force[2 * n + j], -g[2]);
      fi[0] += g[0];
      fi[1] += g[1];
      fi[2] += g[2];
      wv[0] -= av[0] * g[0];
      wv[1] -= av[1] * g[1];
      wv[2] -= av[2] * g[2];
      wv[3] -= av[0] * g[1];
      wv[4] -= av[0] * g[2];
      wv[5] -= av[1] * g[2];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) fi[q] = md_wave_sum(fi[q]);
    if (lane == 0) {
      atomicAdd(&force[i], fi[0]);
      atomicAdd(&force[n + i], fi[1]);
      atomicAdd(&force[2 * n + i], fi[2]);
      acc[0] += e_buf[i];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[1 + q] += wv[q];
    __builtin_amdgcn_wave_barrier();
  }
  if (ev) block_record_add(acc, red, ev + (size_t)(ctl->step % ev_cap) * b.n_rep * MD_EV_LEN,
                           T.rep);
}

// Zero the forces and the record slot of the step being evaluated.
__global__ void k_bpnn_zero(md_batch b, double* force, long long* ev, int ev_cap,
                            const md_ctl_dev* ctl) {
  const size_t n3 = (size_t)3 * b.n_atoms;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n3;
       k += (size_t)gridDim.x * blockDim.x)
    force[k] = 0.0;
  if (ev && blockIdx.x == 0) {
    long long* slot = ev + (size_t)(ctl->step_next % ev_cap) * b.n_rep * MD_EV_LEN;
    for (int q = threadIdx.x; q < b.n_rep * MD_EV_LEN; q += blockDim.x) slot[q] = 0;
  }
}

// Trailing half kick v += half_dt f/m and the kinetic energy into the record.
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_bpnn_kick(md_batch b, const double* force,
                                                             double* vel, double c, double inv_mass,
                                                             long long* ev, int ev_cap,
                                                             const md_ctl_dev* ctl) {
  const int n = b.n_atoms;
  const int lane = threadIdx.x & (MD_WAVE - 1);
  const int tile = blockIdx.x * (MD_ATOM_BLOCK / MD_WAVE) + threadIdx.x / MD_WAVE;
  double k = 0.0;
  int rep = -1;
  if (tile < b.n_tiles) {
    const md_tile T = b.tiles[tile];
    rep = T.rep;
    if (lane < T.count) {
      const int i = T.first + lane;
      double v[3];
      for (int q = 0; q < 3; ++q) {
        v[q] = vel[(size_t)q * n + i] + c * force[(size_t)q * n + i];
        vel[(size_t)q * n + i] = v[q];
      }
      k = 0.5 / (inv_mass * MD_ACCEL) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
  }
  k = md_wave_sum(k);
  if (ev && lane == 0 && rep >= 0)
    atomicAdd((unsigned long long*)&ev[((size_t)(ctl->step % ev_cap) * b.n_rep + rep) * MD_EV_LEN + 7],
              (unsigned long long)(long long)rint(k * MD_EV_SCALE));
}

int load_params(const md_bpnn* p, BpnnDev* d) {
  *d = BpnnDev{};
  if (!p || !p->weights || !(p->r_cut > 0.0) || p->n_g2 < 0 || p->n_g4 < 0 ||
      p->n_g2 + p->n_g4 < 1 || p->n_g2 + p->n_g4 > MD_BPNN_MAX_G || p->h1 < 1 || p->h2 < 1 ||
      p->h1 > MD_BPNN_MAX_HIDDEN || p->h2 > MD_BPNN_MAX_HIDDEN)
    return MD_ERR_ARG;
  d->rc = p->r_cut;
  d->rc2 = p->r_cut * p->r_cut;
  d->rs = p->r_s;
  d->n2 = p->n_g2;
  d->n4 = p->n_g4;
  d->ng = p->n_g2 + p->n_g4;
  d->h1 = p->h1;
  d->h2 = p->h2;
  d->w = p->weights;
  for (int q = 0; q < p->n_g2; ++q) d->g2_eta[q] = p->g2_eta[q];
  for (int q = 0; q < p->n_g4; ++q) {
    const double eta = p->g4_eta[q], zeta = p->g4_zeta[q], lam = p->g4_lambda[q];
    if (!(zeta >= 1.0) || !(lam == 1.0 || lam == -1.0) || !isfinite(eta)) return MD_ERR_ARG;
    int u = 0;
    while (u < d->n_eta && d->eta_u[u] != eta) ++u;
    if (u == d->n_eta) {
      if (u == NE) return MD_ERR_ARG;
      d->eta_u[d->n_eta++] = eta;
    }
    int v = 0;
    while (v < d->n_zl && !(d->zeta_v[v] == zeta && d->lam_v[v] == lam)) ++v;
    if (v == d->n_zl) {
      if (v == NZ) return MD_ERR_ARG;
      d->zeta_v[v] = zeta;
      d->lam_v[v] = lam;
      d->izeta_v[v] = (zeta == floor(zeta) && zeta <= 1024.0) ? (int)zeta : 0;
      ++d->n_zl;
    }
    d->u_of[q] = (unsigned char)u;
    d->v_of[q] = (unsigned char)v;
    d->pref[q] = pow(2.0, 1.0 - zeta);
  }
  return MD_OK;
}

}  // namespace

extern "C" size_t md_bpnn_workspace_bytes(const md_batch* b, const md_bpnn* p) {
  if (!b || !p || p->n_g2 + p->n_g4 < 1) return 0;
  return md_align256((size_t)b->n_atoms * (size_t)(p->n_g2 + p->n_g4 + 1) * sizeof(double));
}

extern "C" int md_bpnn_forces(const md_batch* b, const md_bpnn* p, const double* pos,
                              const md_nlist* nl, double* force, double* e_atom, double* vel,
                              double inv_mass, double half_dt, long long* ev, int ev_cap,
                              void* ws, void* ctl, void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if (!pos || !nl || !nl->neigh || !nl->nneigh || !force || !ws || !ctl) return MD_ERR_ARG;
  if (nl->lanes < 1 || nl->lanes > MD_MAX_LANES || nl->max_neigh < nl->lanes) return MD_ERR_ARG;
  if (ev && ev_cap < 1) return MD_ERR_ARG;
  if (vel && !(inv_mass > 0.0)) return MD_ERR_ARG;
  BpnnDev P;
  if (load_params(p, &P) != MD_OK) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  hipStream_t st = (hipStream_t)stream;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  const size_t npad = (size_t)md_npad(b->n_atoms);
  double* dEdG = (double*)ws;
  double* e_buf = e_atom ? e_atom : dEdG + (size_t)b->n_atoms * P.ng;
  hipLaunchKernelGGL(k_bpnn_zero, dim3(1024), dim3(256), 0, st, *b, force, (long long*)ev, ev_cap,
                     c);
  MD_LAUNCH_CHECK();
  if (P.n_eta <= 6)
    MD_LAUNCH_TIMED(MD_KERNEL_BPNN_DESC, k_bpnn_desc<6>, dim3(b->n_tiles), dim3(64 * WPB), 0, st,
                    *b, P, (const double4*)pos, *nl, npad, dEdG, e_buf, c);
  else
    MD_LAUNCH_TIMED(MD_KERNEL_BPNN_DESC, k_bpnn_desc<NE>, dim3(b->n_tiles), dim3(64 * WPB), 0, st,
                    *b, P, (const double4*)pos, *nl, npad, dEdG, e_buf, c);
  MD_LAUNCH_CHECK();
  MD_LAUNCH_TIMED(MD_KERNEL_BPNN_FORCE, k_bpnn_force, dim3(b->n_tiles), dim3(64 * WPB), 0, st, *b,
                  P, (const double4*)pos, *nl, npad, (const double*)dEdG, (const double*)e_buf,
                  force, (long long*)ev, ev_cap, c);
  MD_LAUNCH_CHECK();
  if (vel) {
    const int nb = (b->n_tiles + MD_ATOM_BLOCK / MD_WAVE - 1) / (MD_ATOM_BLOCK / MD_WAVE);
    hipLaunchKernelGGL(k_bpnn_kick, dim3(nb), dim3(MD_ATOM_BLOCK), 0, st, *b,
                       (const double*)force, vel, half_dt * inv_mass * MD_ACCEL, inv_mass,
                       (long long*)ev, ev_cap, c);
    MD_LAUNCH_CHECK();
  }
  return MD_OK;
}
