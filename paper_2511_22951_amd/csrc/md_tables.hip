// Tabulated potentials on the device: complete cubic spline fit of sampled
// functions and conversion of B-spline coefficients into per-interval
// polynomial tables (the form the force kernels read).
#include "md_internal.h"
#include "md_tables.h"

namespace {

#define MD_FIT_KMAX 8000

// Complete (clamped) cubic interpolation in the uniform B-spline basis.  With
// coefficients c_0..c_{K+1}, s(x_k) = (c_k + 4 c_{k+1} + c_{k+2}) / 6 and
// s'(x_k) = (c_{k+2} - c_k) / (2h).  The two slope conditions eliminate c_0 and
// c_{K+1}; the remaining system for c_1..c_K is tridiagonal and diagonally
// dominant, solved by forward elimination and back substitution.
__global__ void k_spline_fit(const double* y, int K, double h, double dy_lo, double dy_hi,
                             double* coef) {
  __shared__ double cp[MD_FIT_KMAX];
  if (threadIdx.x != 0) return;
  // unknown u_r = c_r, r = 1..K; row r: a_r u_{r-1} + 4 u_r + g_r u_{r+1} = q_r
  double* dp = coef + 1;  // forward-sweep right-hand sides live in the output
  {
    const double g = 2.0, q = 6.0 * y[0] + 2.0 * h * dy_lo;
    cp[0] = g / 4.0;
    dp[0] = q / 4.0;
  }
  for (int r = 2; r <= K; ++r) {
    const double a = (r == K) ? 2.0 : 1.0;
    const double g = (r == K) ? 0.0 : 1.0;
    const double q = (r == K) ? 6.0 * y[K - 1] - 2.0 * h * dy_hi : 6.0 * y[r - 1];
    const double m = 4.0 - a * cp[r - 2];
    cp[r - 1] = g / m;
    dp[r - 1] = (q - a * dp[r - 2]) / m;
  }
  for (int r = K - 1; r >= 1; --r) dp[r - 1] = dp[r - 1] - cp[r - 1] * dp[r];
  coef[0] = coef[2] - 2.0 * h * dy_lo;
  coef[K + 1] = coef[K - 1] + 2.0 * h * dy_hi;
}

// Power-basis coefficients of the B-spline on interval k: s = a0 + a1 t + a2 t^2 + a3 t^3.
__device__ __forceinline__ void interval_poly(const double* c, double a[4]) {
  const double c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
  a[0] = (c0 + 4.0 * c1 + c2) / 6.0;
  a[1] = 0.5 * (c2 - c0);
  a[2] = 0.5 * (c0 - 2.0 * c1 + c2);
  a[3] = (-c0 + 3.0 * c1 - 3.0 * c2 + c3) / 6.0;
}

template <typename R>
__global__ void k_eam_prepare(md_eam p, R* rtab, R* ftab, R* etab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = p.rho.ncoef - 3, ne = p.emb.ncoef - 3;
  if (rtab && k < nr) {
    double ar[4], ap[4];
    interval_poly(p.rho.coef + k, ar);
    interval_poly(p.phi.coef + k, ap);
    const double h = p.rho.h;
    R* d = rtab + (size_t)k * MD_RTAB_W;
    d[0] = (R)ar[0]; d[1] = (R)ar[1]; d[2] = (R)ar[2]; d[3] = (R)ar[3];
    d[4] = (R)ap[0]; d[5] = (R)ap[1]; d[6] = (R)ap[2]; d[7] = (R)ap[3];
    R* f = ftab + (size_t)k * MD_FTAB_W;
    f[0] = (R)(ap[1] / h); f[1] = (R)(2.0 * ap[2] / h); f[2] = (R)(3.0 * ap[3] / h);
    f[3] = (R)(ar[1] / h); f[4] = (R)(2.0 * ar[2] / h); f[5] = (R)(3.0 * ar[3] / h);
    f[6] = (R)0; f[7] = (R)0;
  }
  if (k < ne) {
    double a[4];
    interval_poly(p.emb.coef + k, a);
    const double h = p.emb.h;
    R* e = etab + (size_t)k * MD_ETAB_W;
    e[0] = (R)a[0]; e[1] = (R)a[1]; e[2] = (R)a[2]; e[3] = (R)a[3];
    e[4] = (R)(a[1] / h); e[5] = (R)(2.0 * a[2] / h); e[6] = (R)(3.0 * a[3] / h);
    e[7] = (R)(2.0 * a[2] / (h * h)); e[8] = (R)(6.0 * a[3] / (h * h));
    for (int m = 9; m < MD_ETAB_W; ++m) e[m] = (R)0;
  }
}

// Value, first and second derivative in r of the B-spline (coefficients c,
// breakpoints x_lo + k h, nint intervals) at r; the end intervals extend beyond.
__device__ void spline_eval(const double* c, double x_lo, double h, int nint, double r,
                            double& v, double& d1, double& d2) {
  const double u = (r - x_lo) / h;
  int k = (int)floor(u);
  k = k < 0 ? 0 : (k > nint - 1 ? nint - 1 : k);
  const double t = u - k;
  double a[4];
  interval_poly(c + k, a);
  v = ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
  d1 = ((3.0 * a[3] * t + 2.0 * a[2]) * t + a[1]) / h;
  d2 = (6.0 * a[3] * t + 2.0 * a[2]) / (h * h);
}

// Cubic in t on [0, 1] with values f0, f1 and t-derivatives g0, g1 at the ends.
__device__ void hermite(double f0, double g0, double f1, double g1, float* a) {
  a[0] = (float)f0;
  a[1] = (float)g0;
  a[2] = (float)(3.0 * (f1 - f0) - 2.0 * g0 - g1);
  a[3] = (float)(2.0 * (f0 - f1) + g0 + g1);
}

// FP32 pair tables on the r^2 grid (one thread per interval).  At q = r^2:
// d/dq s(r) = s'(r) / (2 r), and for G = s'(r) / r, dG/dq = (r s'' - s') / (2 r^3).
__global__ void k_eam_prepare_q(md_eam p, double q_lo, double h_q, float* rtab, float* ftab) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= MD_STAB_ROWS) return;
  if (k == MD_STAB_N) {  // beyond r_cut: zero
    for (int m = 0; m < MD_RTAB_W; ++m) rtab[(size_t)k * MD_RTAB_W + m] = 0.0f;
    for (int m = 0; m < MD_FTAB_W; ++m) ftab[(size_t)k * MD_FTAB_W + m] = 0.0f;
    return;
  }
  const int nr = p.rho.ncoef - 3;
  double val[2][2], dq[2][2], G[2][2], dG[2][2];  // [end][phi, rho]
  for (int e = 0; e < 2; ++e) {
    const double q = q_lo + (k + e) * h_q, r = sqrt(q);
    const md_spline* f[2] = {&p.phi, &p.rho};
    for (int m = 0; m < 2; ++m) {
      double v, d1, d2;
      spline_eval(f[m]->coef, f[m]->x_lo, f[m]->h, nr, r, v, d1, d2);
      val[e][m] = v;
      dq[e][m] = d1 / (2.0 * r) * h_q;
      G[e][m] = d1 / r;
      dG[e][m] = (r * d2 - d1) / (2.0 * r * r * r) * h_q;
    }
  }
  float* d = rtab + (size_t)k * MD_RTAB_W;
  hermite(val[0][1], dq[0][1], val[1][1], dq[1][1], d);      // rho
  hermite(val[0][0], dq[0][0], val[1][0], dq[1][0], d + 4);  // phi
  float* f = ftab + (size_t)k * MD_FTAB_W;
  hermite(G[0][0], dG[0][0], G[1][0], dG[1][0], f);      // phi' / r
  hermite(G[0][1], dG[0][1], G[1][1], dG[1][1], f + 4);  // rho' / r
}

}  // namespace

md_qgrid md_qgrid_plan(const md_eam* p) {
  md_qgrid g;
  g.q_lo = p->rho.x_lo * p->rho.x_lo;
  g.h = (p->r_cut * p->r_cut - g.q_lo) / MD_STAB_N;
  return g;
}

md_table_layout md_table_plan(const md_eam* p, md_precision prec) {
  md_table_layout L;
  const size_t es = prec == MD_FP32 ? 4 : 8;
  const size_t ne = (size_t)(p->emb.ncoef - 3);
  const size_t nr = prec == MD_FP32 ? (size_t)MD_STAB_ROWS : (size_t)(p->rho.ncoef - 3);
  L.rtab = 0;
  L.ftab = md_align256(nr * MD_RTAB_W * es);
  L.etab = L.ftab + md_align256(nr * MD_FTAB_W * es);
  L.total = L.etab + md_align256(ne * MD_ETAB_W * es);
  return L;
}

bool md_eam_ok(const md_eam* p) {
  if (!p) return false;
  const md_spline* s[3] = {&p->phi, &p->rho, &p->emb};
  for (int k = 0; k < 3; ++k)
    if (!s[k]->coef || s[k]->ncoef < 6 || !(s[k]->h > 0.0)) return false;
  // phi and rho share one grid (one interval lookup serves both)
  if (p->phi.ncoef != p->rho.ncoef || p->phi.x_lo != p->rho.x_lo || p->phi.h != p->rho.h)
    return false;
  if (!(p->r_cut > p->rho.x_lo)) return false;
  // the table must reach the cutoff
  if (p->rho.x_lo + (p->rho.ncoef - 3) * p->rho.h < p->r_cut * (1.0 - 1e-12)) return false;
  return true;
}

extern "C" size_t md_eam_table_bytes(const md_eam* p, md_precision prec) {
  if (!md_eam_ok(p)) return 0;
  return md_table_plan(p, prec).total;
}

extern "C" int md_spline_fit(const double* y, int K, double h, double dy_lo, double dy_hi,
                             double* coef, void* stream) {
  if (!y || !coef || K < 4 || K > MD_FIT_KMAX || !(h > 0.0)) return MD_ERR_ARG;
  hipLaunchKernelGGL(k_spline_fit, dim3(1), dim3(64), 0, (hipStream_t)stream, y, K, h, dy_lo,
                     dy_hi, coef);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" int md_eam_prepare(const md_eam* p, md_precision prec, void* table, void* stream) {
  if (!md_eam_ok(p) || !table || (prec != MD_FP64 && prec != MD_FP32)) return MD_ERR_ARG;
  const md_table_layout L = md_table_plan(p, prec);
  const int n = p->rho.ncoef > p->emb.ncoef ? p->rho.ncoef : p->emb.ncoef;
  const dim3 grid((n + 255) / 256), block(256);
  char* t = (char*)table;
  if (prec == MD_FP32) {
    // embedding rows from the rhobar spline; pair rows resampled on the r^2 grid
    hipLaunchKernelGGL(k_eam_prepare<float>, grid, block, 0, (hipStream_t)stream, *p,
                       (float*)nullptr, (float*)nullptr, (float*)(t + L.etab));
    MD_LAUNCH_CHECK();
    const md_qgrid q = md_qgrid_plan(p);
    hipLaunchKernelGGL(k_eam_prepare_q, dim3((MD_STAB_ROWS + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, *p, q.q_lo, q.h, (float*)(t + L.rtab),
                       (float*)(t + L.ftab));
  } else
    hipLaunchKernelGGL(k_eam_prepare<double>, grid, block, 0, (hipStream_t)stream, *p,
                       (double*)(t + L.rtab), (double*)(t + L.ftab), (double*)(t + L.etab));
  MD_LAUNCH_CHECK();
  return MD_OK;
}
