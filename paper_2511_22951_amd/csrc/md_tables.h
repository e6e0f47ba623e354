// Packed EAM interval tables (written by md_eam_prepare, read by the force kernels).
//
// For a function s with B-spline coefficients c on breakpoints x_lo + k h, the
// interval k (x_k <= x < x_{k+1}, t = (x - x_k) / h) is the cubic
// s = a0 + a1 t + a2 t^2 + a3 t^3.  Rows, in the table precision:
//   rtab[k][8]  = {rho a0..a3, phi a0..a3}                 (density pass: values)
//   ftab[k][8]  = {phi' d0..d2, rho' d0..d2, 0, 0}          (force pass: s' = d0 + d1 t + d2 t^2)
//   etab[k][16] = {F a0..a3, F' d0..d2, F'' e0, e1, 0...}   (embedding: F'' = e0 + e1 t)
#pragma once

#include "md.h"

#define MD_RTAB_W 8
#define MD_FTAB_W 8
#define MD_ETAB_W 16

struct md_table_layout {
  size_t rtab, ftab, etab, total;
};

md_table_layout md_table_plan(const md_eam* p, md_precision prec);
bool md_eam_ok(const md_eam* p);
