// Packed EAM interval tables (written by md_eam_prepare, read by the force kernels).
//
// FP64: for a function s with B-spline coefficients c on breakpoints x_lo + k h,
// the interval k (x_k <= x < x_{k+1}, t = (x - x_k) / h) is the cubic
// s = a0 + a1 t + a2 t^2 + a3 t^3.  Rows:
//   rtab[k][8]  = {rho a0..a3, phi a0..a3}                 (density pass: values)
//   ftab[k][8]  = {phi' d0..d2, rho' d0..d2, 0, 0}          (force pass: s' = d0 + d1 t + d2 t^2)
//   etab[k][16] = {F a0..a3, F' d0..d2, F'' e0, e1, 0...}   (embedding: F'' = e0 + e1 t)
//
// FP32 pair tables are indexed by the squared distance instead, so that the pair
// loops need no square root: MD_STAB_N intervals of a uniform grid in q = r^2 on
// [x_lo^2, r_cut^2], each a cubic in t = (q - q_k) / h_q, the Hermite interpolant
// of the spline's values and q-derivatives at the interval ends (resampled in
// FP64; interpolation error ~1e-10 relative for the 2000-point tables):
//   rtab[k][8] = {rho a0..a3, phi a0..a3}
//   ftab[k][8] = {phi'/r a0..a3, rho'/r a0..a3}            (G(q) = s'(r) / r)
// followed by one row of zeros (k = MD_STAB_N): the pair loops clamp every q beyond
// r_cut^2 onto it, so that pairs past the cutoff add exactly zero without a compare.
// The embedding table stays on the rhobar grid as above.
#pragma once

#include "md.h"

#define MD_RTAB_W 8
#define MD_FTAB_W 8
#define MD_ETAB_W 16
#define MD_STAB_N 2000  // FP32 pair tables: intervals in r^2 (2000 x 32 B fits 64 KB of LDS)
#define MD_STAB_ROWS (MD_STAB_N + 1)  // FP32 pair-table rows: the intervals and the zero row

struct md_table_layout {
  size_t rtab, ftab, etab, total;
};

md_table_layout md_table_plan(const md_eam* p, md_precision prec);

// The r^2 grid of the FP32 pair tables: q_k = q_lo + k h, k = 0..MD_STAB_N.
struct md_qgrid {
  double q_lo, h;
};
md_qgrid md_qgrid_plan(const md_eam* p);
bool md_eam_ok(const md_eam* p);
