// Velocity Verlet (Sec. 1.5): kick-drift with walls and the neighbour-list
// displacement check, and the stand-alone half kick.
#include <math.h>

#include "md_internal.h"

namespace {

struct Walls {
  int enabled, axis;
  double z0, v, top;
};

// v += dt/2 f/m; x += dt v; walls at t = (step + 1) dt; per-block maximum of
// |x - x_ref|^2 into ctl->dmax[blockIdx.x].
template <typename R>
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_kick_drift(
    md_batch b, double dt, double half_dt, double4* pos, double* vel, const R* force,
    double inv_mass, Walls w, const double* pos_ref, double thr2, md_ctl_dev* ctl) {
  __shared__ double sh[MD_ATOM_BLOCK / MD_WAVE];
  const int nlb = (b.n_tiles + 3) / 4;
  const int lane = threadIdx.x & (MD_WAVE - 1);
  const int n = b.n_atoms;
  const double t_new = (double)(ctl->step + 1) * dt;
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
    double v[3] = {vel[i] + c * (double)force[i], vel[n + i] + c * (double)force[n + i],
                   vel[2 * n + i] + c * (double)force[2 * n + i]};
    const double4 p = pos[i];
    double x[3] = {p.x + dt * v[0], p.y + dt * v[1], p.z + dt * v[2]};
    if (w.enabled) {
      const int a = w.axis;
      const double zp = w.z0 + w.v * t_new;
      if (x[a] < zp) {  // specular reflection in the piston frame
        x[a] = 2.0 * zp - x[a];
        v[a] = 2.0 * w.v - v[a];
      }
      if (x[a] > w.top) {
        x[a] = 2.0 * w.top - x[a];
        v[a] = -v[a];
      }
    }
    vel[i] = v[0];
    vel[n + i] = v[1];
    vel[2 * n + i] = v[2];
    pos[i] = make_double4(x[0], x[1], x[2], p.w);
    if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2])) bad |= MD_FLAG_NONFINITE;
    const double dx = x[0] - pos_ref[i], dy = x[1] - pos_ref[n + i], dz = x[2] - pos_ref[2 * n + i];
    double d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 >= 0.0)) d2 = INFINITY;  // NaN forces a rebuild (and is flagged)
    d2max = fmax(d2max, d2);
  }
#pragma unroll
  for (int o = MD_WAVE / 2; o > 0; o >>= 1) d2max = fmax(d2max, __shfl_xor(d2max, o, MD_WAVE));
  if (__any(bad)) {
    int all = bad;
#pragma unroll
    for (int o = MD_WAVE / 2; o > 0; o >>= 1) all |= __shfl_xor(all, o, MD_WAVE);
    if (lane == 0) md_flag(ctl, all);
  }
  if (lane == 0) sh[threadIdx.x / MD_WAVE] = d2max;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int k = 1; k < MD_ATOM_BLOCK / MD_WAVE; ++k) m = fmax(m, sh[k]);
    ctl->dmax[blockIdx.x] = m;
    if (blockIdx.x == 0) {  // fields no block of this kernel reads
      ctl->n_dmax = gridDim.x;
      ctl->thr2 = thr2;
      ctl->step_next = ctl->step + 1;
    }
  }
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
    vel[i] += c * (double)force[i];
    vel[n + i] += c * (double)force[n + i];
    vel[2 * n + i] += c * (double)force[2 * n + i];
  }
}

}  // namespace

extern "C" int md_verlet_step(const md_batch* b, md_verlet_phase phase, double dt, double* pos,
                              double* vel, const void* force, md_precision prec, double inv_mass,
                              const md_walls* walls, const double* pos_ref, double half_skin,
                              void* ctl, void* stream) {
  if (!b || b->n_rep < 1 || !b->tiles || !b->domains || b->tile_atoms != MD_TILE) return MD_ERR_ARG;
  if (!vel || !force || !(inv_mass > 0.0) || !isfinite(dt)) return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (b->n_atoms == 0) return MD_OK;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid(md_atom_grid(b->n_tiles)), block(MD_ATOM_BLOCK);
  if (phase == MD_KICK) {
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
  Walls w{0, 2, 0.0, 0.0, 0.0};
  if (walls && walls->enabled) {
    if (walls->axis < 0 || walls->axis > 2) return MD_ERR_ARG;
    w.enabled = 1;
    w.axis = walls->axis;
    w.z0 = walls->piston_z0;
    w.v = walls->piston_v;
    w.top = walls->top;
  }
  const double thr2 = half_skin < 0.0 ? -1.0 : half_skin * half_skin;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  if (prec == MD_FP32)
    MD_LAUNCH_TIMED(MD_KERNEL_KICK_DRIFT, k_kick_drift<float>, grid, block, 0, st, *b, dt,
                    0.5 * dt, (double4*)pos, vel, (const float*)force, inv_mass, w, pos_ref, thr2, c);
  else
    MD_LAUNCH_TIMED(MD_KERNEL_KICK_DRIFT, k_kick_drift<double>, grid, block, 0, st, *b, dt,
                    0.5 * dt, (double4*)pos, vel, (const double*)force, inv_mass, w, pos_ref, thr2, c);
  MD_LAUNCH_CHECK();
  return MD_OK;
}
