// Velocity Verlet (Sec. 1.5): kick-drift with walls and the neighbour-list
// displacement check, and the stand-alone half kick.
#include <math.h>

#include "md_internal.h"

namespace {

// THERMO: the Langevin update; then v += dt/2 f/m; x += dt v; walls at
// t = (step + 1) dt; per-block maximum of |x - x_ref|^2 into ctl->dmax[blockIdx.x].
template <typename R, bool THERMO>
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_kick_drift(
    md_batch b, double dt, double half_dt, double4* pos, double* vel, const R* force,
    double inv_mass, md_walls_dev w, md_langevin_dev L, const double* pos_ref, double thr2,
    md_ctl_dev* ctl) {
  const int nlb = (b.n_tiles + 3) / 4;
  const int lane = threadIdx.x & (MD_WAVE - 1);
  const int n = b.n_atoms;
  const int step = ctl->step + 1;
  const double t_new = (double)step * dt;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->rec_stale = 1;  // positions move here
  const double c = half_dt * inv_mass * MD_ACCEL;
  double d2max = 0.0;
  int bad = 0;
  for (int k = 0;; ++k) {
    const int lb = md_remap_stride(nlb, k);
    if (lb >= nlb) break;
    const int tile = lb * 4 + (int)(threadIdx.x / MD_WAVE);
    if (tile >= b.n_tiles) continue;
    const md_tile T = b.tiles[tile];
    if (lane >= T.count) continue;
    const int i = T.first + lane;
    const double4 p = pos[i];
    double x[3] = {p.x, p.y, p.z};
    double v[3];
    if (THERMO) {
      v[0] = vel[i];
      v[1] = vel[n + i];
      v[2] = vel[2 * n + i];
      md_langevin_atom(L, b.domains[T.rep], i, step, x, v);
      v[0] = md_kick(v[0], c, (double)force[i]);
      v[1] = md_kick(v[1], c, (double)force[n + i]);
      v[2] = md_kick(v[2], c, (double)force[2 * n + i]);
    } else {
      v[0] = md_kick(vel[i], c, (double)force[i]);
      v[1] = md_kick(vel[n + i], c, (double)force[n + i]);
      v[2] = md_kick(vel[2 * n + i], c, (double)force[2 * n + i]);
    }
    md_drift_atom(x, v, dt, w, t_new);
    vel[i] = v[0];
    vel[n + i] = v[1];
    vel[2 * n + i] = v[2];
    pos[i] = make_double4(x[0], x[1], x[2], p.w);
    if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2])) bad |= MD_FLAG_NONFINITE;
    d2max = fmax(d2max, md_disp2(x, pos_ref, i, n));
  }
  md_publish_dmax(d2max, bad, thr2, ctl);
}

template <typename R>
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_kick(md_batch b, double half_dt, double* vel,
                                                        const R* force, double inv_mass) {
  const int nlb = (b.n_tiles + 3) / 4;
  const int lane = threadIdx.x & (MD_WAVE - 1), n = b.n_atoms;
  const double c = half_dt * inv_mass * MD_ACCEL;
  for (int k = 0;; ++k) {
    const int lb = md_remap_stride(nlb, k);
    if (lb >= nlb) break;
    const int tile = lb * 4 + (int)(threadIdx.x / MD_WAVE);
    if (tile >= b.n_tiles) continue;
    const md_tile T = b.tiles[tile];
    if (lane >= T.count) continue;
    const int i = T.first + lane;
    vel[i] = md_kick(vel[i], c, (double)force[i]);
    vel[n + i] = md_kick(vel[n + i], c, (double)force[n + i]);
    vel[2 * n + i] = md_kick(vel[2 * n + i], c, (double)force[2 * n + i]);
  }
}

}  // namespace

// Host form of md_langevin for one time step and mass.
int md_langevin_load(const md_langevin* lg, double dt, double inv_mass, md_langevin_dev* L) {
  *L = md_langevin_dev{};
  if (!lg) return MD_OK;
  if (!lg->id || lg->axis < 0 || lg->axis > 2 || lg->n_regions < 1 ||
      lg->n_regions > MD_MAX_THERMO_REGIONS)
    return MD_ERR_ARG;
  const double kB = 8.617333262e-5;  // eV/K
  L->id = lg->id;
  L->key0 = (unsigned)(lg->seed & 0xFFFFFFFFull);
  L->key1 = (unsigned)(lg->seed >> 32);
  L->axis = lg->axis;
  L->n = lg->n_regions;
  for (int q = 0; q < lg->n_regions; ++q) {
    const md_thermo_region& R = lg->region[q];
    if (!(R.temperature >= 0.0) || !(R.gamma >= 0.0) || isnan(R.lo) || isnan(R.hi))
      return MD_ERR_ARG;
    const double c1 = exp(-R.gamma * dt);
    L->lo[q] = R.lo;
    L->hi[q] = R.hi;
    L->c1[q] = c1;
    L->c2[q] = sqrt((1.0 - c1 * c1) * kB * R.temperature * inv_mass * MD_ACCEL);
    for (int k = 0; k < 3; ++k) {
      if (!isfinite(R.u[k])) return MD_ERR_ARG;
      L->u[q][k] = R.u[k];
    }
  }
  return MD_OK;
}

extern "C" int md_verlet_step(const md_batch* b, md_verlet_phase phase, double dt, double* pos,
                              double* vel, const void* force, md_precision prec, double inv_mass,
                              const md_walls* walls, const md_langevin* lang,
                              const double* pos_ref, double half_skin, void* ctl, void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if (!vel || !force || !(inv_mass > 0.0) || !isfinite(dt)) return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
  if (phase == MD_KICK) {
    if (lang) return MD_ERR_ARG;
    if (prec == MD_FP32)
      hipLaunchKernelGGL(k_kick<float>, grid, block, 0, st, *b, 0.5 * dt, vel,
                         (const float*)force, inv_mass);
    else
      hipLaunchKernelGGL(k_kick<double>, grid, block, 0, st, *b, 0.5 * dt, vel,
                         (const double*)force, inv_mass);
    MD_LAUNCH_CHECK();
    return MD_OK;
  }
  if (phase != MD_KICK_DRIFT || !pos || !pos_ref || !ctl) return MD_ERR_ARG;
  md_walls_dev w;
  if (md_walls_load(walls, &w) != MD_OK) return MD_ERR_ARG;
  md_langevin_dev L;
  if (md_langevin_load(lang, dt, inv_mass, &L) != MD_OK) return MD_ERR_ARG;
  const double thr2 = half_skin < 0.0 ? -1.0 : half_skin * half_skin;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
#define MD_KD_LAUNCH(R, TH)                                                                       \
  MD_LAUNCH_TIMED(MD_KERNEL_KICK_DRIFT, (k_kick_drift<R, TH>), grid, block, 0, st, *b, dt,       \
                  0.5 * dt, (double4*)pos, vel, (const R*)force, inv_mass, w, L, pos_ref, thr2, c)
  if (prec == MD_FP32) {
    if (lang) MD_KD_LAUNCH(float, true);
    else MD_KD_LAUNCH(float, false);
  } else {
    if (lang) MD_KD_LAUNCH(double, true);
    else MD_KD_LAUNCH(double, false);
  }
#undef MD_KD_LAUNCH
  MD_LAUNCH_CHECK();
  return MD_OK;
}
