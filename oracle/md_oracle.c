/*
 * FP64 O(N^2) minimum-image reference for the short-range MD path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: it is compiled into its
 * own shared object, called from the tests, the smoke check and the CPU
 * baseline timing, and never linked into or called by the HIP library.  It
 * shares no code with it.
 *
 * Everything here is the plain definition, written out:
 *   - minimum image on periodic axes, d -= L * rint(d / L);
 *   - the Verlet neighbour set {j != i : r^2 < r_ns^2} (Sec. 1.4, eq. 1.2),
 *     found by brute force over all pairs (the O(N^2) search of Sec. 1.4);
 *   - pair forces f_i = -sum_j V'(r_ij) r_ij / r_ij (Sec. 1.6, eq. 1.6, with
 *     r_ij = x_i - x_j), Lennard-Jones with an energy shift at r_c;
 *   - single-element EAM (Sec. 1.6, Sec. 3.3) in the standard embedded-atom
 *     form E = sum_i F(rhobar_i) + 1/2 sum_{i != j} phi(r_ij),
 *     rhobar_i = sum_{j != i} rho(r_ij), truncated at r_c;
 *   - uniform cubic B-spline evaluation from its definition (basis functions
 *     of the uniform cardinal cubic B-spline), or the analytic closed forms;
 *   - virial W^{ab} = 1/2 sum_i sum_{j != i} r_ij^a f_ij^b (Appendix, read as
 *     the Clausius pair virial).
 * Compiled with -O2 -ffp-contract=off (no fused multiply-add).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  double lo[3];
  double len[3];
  int periodic[3];
} or_box;

/* A 1-D function: either a uniform cubic B-spline (kind 0) with ncoef = K + 2
 * coefficients on breakpoints x_lo + k h, k = 0..K-1, or an analytic closed
 * form (kind 1: A exp(-alpha (x/r0 - 1)); kind 2: -sqrt(x)). */
typedef struct {
  int kind;
  int ncoef;
  const double* c;
  double x_lo;
  double h;
  double A, alpha, r0;
} or_func;

typedef struct {
  or_func phi, rho, emb;
  double r_cut;
} or_eam_pot;

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static void min_image(const or_box* b, double d[3]) {
  for (int a = 0; a < 3; ++a)
    if (b->periodic[a]) d[a] = d[a] - b->len[a] * rint(d[a] / b->len[a]);
}

/* r_ij = x_i - x_j under the minimum image; returns r^2 = (x*x + y*y) + z*z. */
static double sep(const or_box* b, const double* xi, const double* xj, double rij[3]) {
  double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
  min_image(b, d);
  rij[0] = -d[0];
  rij[1] = -d[1];
  rij[2] = -d[2];
  return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* Wrap: x <- x - L floor((x - lo) / L) on periodic axes; a result equal to
 * lo + L (rounding) is set to lo. */
void or_wrap(int n, double* pos, const or_box* b) {
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      if (!b->periodic[a]) continue;
      double x = pos[3 * i + a];
      x = x - b->len[a] * floor((x - b->lo[a]) / b->len[a]);
      if (x >= b->lo[a] + b->len[a]) x = b->lo[a];
      pos[3 * i + a] = x;
    }
}

/* Brute-force neighbour sets, ascending j.  Returns the number of atoms whose
 * set exceeded maxn (their lists are truncated, counts are exact). */
int or_neighbors(int n, const double* pos, const or_box* b, double r_ns, int maxn, int* cnt,
                 int* list) {
  const double rns2 = r_ns * r_ns;
  int over = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : over)
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
      if (r2 < rns2) {
        if (c < maxn) list[(size_t)i * maxn + c] = j;
        ++c;
      }
    }
    cnt[i] = c;
    if (c > maxn) ++over;
  }
  return over;
}

/* Smallest |r - r_probe| over all pairs (used by tests to show that no pair sits
 * on a comparison boundary). */
double or_min_gap(int n, const double* pos, const or_box* b, double r_probe) {
  double best = INFINITY;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : best)
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double rij[3];
      double r = sqrt(sep(b, pos + 3 * i, pos + 3 * j, rij));
      double g = fabs(r - r_probe);
      if (g < best) best = g;
    }
  return best;
}

/* ---------------------------------------------------------------------------
 * Lennard-Jones, U(r) = 4 eps [(s/r)^12 - (s/r)^6] - U(r_c) for r < r_c.
 * Outputs per-atom force [n][3], energy [n] (half of each pair) and virial
 * [n][6] (xx, yy, zz, xy, xz, yz; half of each pair).
 * ------------------------------------------------------------------------- */
void or_lj(int n, const double* pos, const or_box* b, double eps, double sigma, double r_cut,
           double* f, double* e_atom, double* w_atom) {
  const double rc2 = r_cut * r_cut;
  const double src6 = pow(sigma / r_cut, 6.0);
  const double u_cut = 4.0 * eps * (src6 * src6 - src6);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) {
    double fi[3] = {0, 0, 0}, ei = 0.0, wi[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
      if (!(r2 < rc2)) continue;
      double sr2 = sigma * sigma / r2;
      double sr6 = sr2 * sr2 * sr2;
      double sr12 = sr6 * sr6;
      double u = 4.0 * eps * (sr12 - sr6) - u_cut;
      /* -dU/dr / r */
      double fs = 24.0 * eps * (2.0 * sr12 - sr6) / r2;
      double fij[3] = {fs * rij[0], fs * rij[1], fs * rij[2]};
      for (int a = 0; a < 3; ++a) fi[a] += fij[a];
      ei += 0.5 * u;
      wi[0] += 0.5 * rij[0] * fij[0];
      wi[1] += 0.5 * rij[1] * fij[1];
      wi[2] += 0.5 * rij[2] * fij[2];
      wi[3] += 0.5 * rij[0] * fij[1];
      wi[4] += 0.5 * rij[0] * fij[2];
      wi[5] += 0.5 * rij[1] * fij[2];
    }
    for (int a = 0; a < 3; ++a) f[3 * i + a] = fi[a];
    e_atom[i] = ei;
    for (int k = 0; k < 6; ++k) w_atom[6 * i + k] = wi[k];
  }
}

/* ---------------------------------------------------------------------------
 * Uniform cubic B-spline: u = (x - x_lo)/h, i = clamp(floor(u), 0, K-2),
 * t = u - i, s(x) = sum_m c[i+m] b_m(t) with the cardinal cubic basis
 *   b0 = (1-t)^3/6, b1 = (3t^3 - 6t^2 + 4)/6, b2 = (-3t^3 + 3t^2 + 3t + 1)/6,
 *   b3 = t^3/6.
 * Returns 1 when x lies outside [x_lo, x_lo + (K-1) h] (the end interval's
 * polynomial is used there).
 * ------------------------------------------------------------------------- */
static int eval_func(const or_func* fn, double x, double* v, double* d1, double* d2) {
  if (fn->kind == 1) {
    double e = fn->A * exp(-fn->alpha * (x / fn->r0 - 1.0));
    double k = -fn->alpha / fn->r0;
    *v = e;
    *d1 = k * e;
    *d2 = k * k * e;
    return 0;
  }
  if (fn->kind == 2) {
    double s = sqrt(x);
    *v = -s;
    *d1 = -0.5 / s;
    *d2 = 0.25 / (s * x);
    return x <= 0.0;
  }
  const int K = fn->ncoef - 2;
  const double u = (x - fn->x_lo) / fn->h;
  int oor = (u < 0.0) || (u > (double)(K - 1));
  double fl = floor(u);
  int i = (int)fl;
  if (fl < 0.0) i = 0;
  if (fl > (double)(K - 2)) i = K - 2;
  const double t = u - (double)i;
  const double s = 1.0 - t;
  const double b0 = s * s * s / 6.0;
  const double b1 = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  const double b2 = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  const double b3 = t * t * t / 6.0;
  const double g0 = -0.5 * s * s;
  const double g1 = (3.0 * t * t - 4.0 * t) / 2.0;
  const double g2 = (-3.0 * t * t + 2.0 * t + 1.0) / 2.0;
  const double g3 = 0.5 * t * t;
  const double h0 = s;
  const double h1 = 3.0 * t - 2.0;
  const double h2 = 1.0 - 3.0 * t;
  const double h3 = t;
  const double* c = fn->c + i;
  *v = c[0] * b0 + c[1] * b1 + c[2] * b2 + c[3] * b3;
  *d1 = (c[0] * g0 + c[1] * g1 + c[2] * g2 + c[3] * g3) / fn->h;
  *d2 = (c[0] * h0 + c[1] * h1 + c[2] * h2 + c[3] * h3) / (fn->h * fn->h);
  return oor;
}

/* Vectorised evaluation for tests of the spline itself. */
int or_eval_func(const or_func* fn, int m, const double* x, double* v, double* d1, double* d2) {
  int oor = 0;
  for (int k = 0; k < m; ++k) oor += eval_func(fn, x[k], v + k, d1 + k, d2 + k);
  return oor;
}

/* ---------------------------------------------------------------------------
 * EAM, all atoms.  Pass 1 (density): rhobar_i, F(rhobar_i), F'(rhobar_i), the
 * per-atom energy F(rhobar_i) + 1/2 sum_j phi(r_ij).  Pass 2 (force):
 *   f_i = -sum_j [phi'(r) + (F'_i + F'_j) rho'(r)] r_ij / r.
 * Per-atom virial as in or_lj.  Returns the number of out-of-table-range
 * evaluations.
 * ------------------------------------------------------------------------- */
int or_eam(int n, const double* pos, const or_box* b, const or_eam_pot* p, double* rhobar,
           double* fp, double* fpp, double* f, double* e_atom, double* w_atom) {
  const double rc2 = p->r_cut * p->r_cut;
  int oor = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : oor)
  for (int i = 0; i < n; ++i) {
    double rb = 0.0, ph = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
      if (!(r2 < rc2)) continue;
      double r = sqrt(r2), v, d1, d2;
      oor += eval_func(&p->rho, r, &v, &d1, &d2);
      rb += v;
      oor += eval_func(&p->phi, r, &v, &d1, &d2);
      ph += v;
    }
    double F, F1, F2;
    oor += eval_func(&p->emb, rb, &F, &F1, &F2);
    rhobar[i] = rb;
    fp[i] = F1;
    if (fpp) fpp[i] = F2;
    e_atom[i] = F + 0.5 * ph;
  }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : oor)
  for (int i = 0; i < n; ++i) {
    double fi[3] = {0, 0, 0}, wi[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
      if (!(r2 < rc2)) continue;
      double r = sqrt(r2), vphi, dphi, vrho, drho, d2;
      oor += eval_func(&p->phi, r, &vphi, &dphi, &d2);
      oor += eval_func(&p->rho, r, &vrho, &drho, &d2);
      double fs = -(dphi + (fp[i] + fp[j]) * drho) / r;
      double fij[3] = {fs * rij[0], fs * rij[1], fs * rij[2]};
      for (int a = 0; a < 3; ++a) fi[a] += fij[a];
      wi[0] += 0.5 * rij[0] * fij[0];
      wi[1] += 0.5 * rij[1] * fij[1];
      wi[2] += 0.5 * rij[2] * fij[2];
      wi[3] += 0.5 * rij[0] * fij[1];
      wi[4] += 0.5 * rij[0] * fij[2];
      wi[5] += 0.5 * rij[1] * fij[2];
    }
    for (int a = 0; a < 3; ++a) f[3 * i + a] = fi[a];
    for (int k = 0; k < 6; ++k) w_atom[6 * i + k] = wi[k];
  }
  return oor;
}

/* rhobar of one atom by brute force. */
static double rhobar_of(int n, const double* pos, const or_box* b, const or_eam_pot* p, int i,
                        int* oor) {
  const double rc2 = p->r_cut * p->r_cut;
  double rb = 0.0;
  for (int j = 0; j < n; ++j) {
    if (j == i) continue;
    double rij[3];
    double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
    if (!(r2 < rc2)) continue;
    double v, d1, d2;
    *oor += eval_func(&p->rho, sqrt(r2), &v, &d1, &d2);
    rb += v;
  }
  return rb;
}

/* EAM on a sample of atoms of a large system: for each sampled atom i its
 * rhobar, energy and force, with rhobar_j of every neighbour recomputed by
 * brute force.  Cost per sample ~ (1 + neighbours) * n pair tests. */
int or_eam_sampled(int n, const double* pos, const or_box* b, const or_eam_pot* p, int ns,
                   const int* idx, double* rhobar_s, double* f_s, double* e_s) {
  const double rc2 = p->r_cut * p->r_cut;
  int oor = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : oor)
  for (int s = 0; s < ns; ++s) {
    const int i = idx[s];
    double rbi = rhobar_of(n, pos, b, p, i, &oor);
    double F, F1i, F2;
    oor += eval_func(&p->emb, rbi, &F, &F1i, &F2);
    double fi[3] = {0, 0, 0}, ph = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
      if (!(r2 < rc2)) continue;
      double rbj = rhobar_of(n, pos, b, p, j, &oor), Fj, F1j, F2j;
      oor += eval_func(&p->emb, rbj, &Fj, &F1j, &F2j);
      double r = sqrt(r2), vphi, dphi, vrho, drho, d2;
      oor += eval_func(&p->phi, r, &vphi, &dphi, &d2);
      oor += eval_func(&p->rho, r, &vrho, &drho, &d2);
      ph += vphi;
      double fs = -(dphi + (F1i + F1j) * drho) / r;
      for (int a = 0; a < 3; ++a) fi[a] += fs * rij[a];
    }
    rhobar_s[s] = rbi;
    e_s[s] = F + 0.5 * ph;
    for (int a = 0; a < 3; ++a) f_s[3 * s + a] = fi[a];
  }
  return oor;
}

/* LJ on a sample of atoms (force and energy of each sampled atom). */
void or_lj_sampled(int n, const double* pos, const or_box* b, double eps, double sigma,
                   double r_cut, int ns, const int* idx, double* f_s, double* e_s) {
  const double rc2 = r_cut * r_cut;
  const double src6 = pow(sigma / r_cut, 6.0);
  const double u_cut = 4.0 * eps * (src6 * src6 - src6);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < ns; ++s) {
    const int i = idx[s];
    double fi[3] = {0, 0, 0}, ei = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      double r2 = sep(b, pos + 3 * i, pos + 3 * j, rij);
      if (!(r2 < rc2)) continue;
      double sr2 = sigma * sigma / r2, sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
      double fs = 24.0 * eps * (2.0 * sr12 - sr6) / r2;
      for (int a = 0; a < 3; ++a) fi[a] += fs * rij[a];
      ei += 0.5 * (4.0 * eps * (sr12 - sr6) - u_cut);
    }
    for (int a = 0; a < 3; ++a) f_s[3 * s + a] = fi[a];
    e_s[s] = ei;
  }
}

/* Neighbour sets of a sample of atoms (ascending j), for large-system parity. */
void or_neighbors_sampled(int n, const double* pos, const or_box* b, double r_ns, int ns,
                          const int* idx, int maxn, int* cnt, int* list) {
  const double rns2 = r_ns * r_ns;
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < ns; ++s) {
    const int i = idx[s];
    int c = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      if (sep(b, pos + 3 * i, pos + 3 * j, rij) < rns2) {
        if (c < maxn) list[(size_t)s * maxn + c] = j;
        ++c;
      }
    }
    cnt[s] = c;
  }
}

/* All pairs (i, j), i != j, with r^2 < r_c^2: arrays of i, j and r_ij
 * (x_i - x_j, minimum image).  Returns the number of pairs found; writes at most
 * cap of them.  Used by the force-matching oracle, whose positions are fixed. */
long or_pairs(int n, const double* pos, const or_box* b, double r_cut, long cap, int* pi, int* pj,
              double* rvec) {
  const double rc2 = r_cut * r_cut;
  long m = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double rij[3];
      if (sep(b, pos + 3 * i, pos + 3 * j, rij) < rc2) {
        if (m < cap) {
          pi[m] = i;
          pj[m] = j;
          rvec[3 * m] = rij[0];
          rvec[3 * m + 1] = rij[1];
          rvec[3 * m + 2] = rij[2];
        }
        ++m;
      }
    }
  return m;
}
