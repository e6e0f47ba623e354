// Force passes over the Verlet list (Sec. 1.6): Lennard-Jones, and the EAM
// density and force passes, with the trailing velocity-Verlet half kick and the
// energy / virial / kinetic-energy reductions fused in.
//
// Mapping: one work tile of 64 consecutive (cell-ordered) atoms per block and
// LANES lanes per atom, so a block has 64 * LANES threads.  Lane l of an atom
// walks list entries l, l + LANES, ...; with the strided ELL layout the LANES
// lanes of 64 / LANES atoms read one contiguous 256-byte segment per step.
// Each atom's force is reduced over its lanes with butterflies and written by
// its first lane: a gather formulation, with no atomics on forces.
//
// Precision R: double (MD_FP64) or float (MD_FP32).  In FP32 the separation
// is formed in FP64 from the FP64 positions and then rounded; pair arithmetic
// and the per-atom force/density sums are FP32; velocities, the kick and all
// block / global reductions are FP64.
#include <math.h>

#include "md_internal.h"
#include "md_tables.h"

namespace {

template <typename R> __device__ __forceinline__ R rsqrt_r(R x);
template <> __device__ __forceinline__ double rsqrt_r<double>(double x) { return rsqrt(x); }
template <> __device__ __forceinline__ float rsqrt_r<float>(float x) { return rsqrtf(x); }

struct TabGeom {
  double r_lo, r_inv_h, e_lo, e_inv_h;
  int nr, ne;  // intervals
};

// Interval index and local coordinate; sets oor when x is below the table.
template <typename R>
__device__ __forceinline__ int tab_index(R x, R lo, R inv_h, int nint, R& t, bool& oor) {
  const R u = (x - lo) * inv_h;
  int k = (int)u;
  if (u < (R)0) {
    oor = true;
    k = 0;
  }
  if (k > nint - 1) k = nint - 1;
  t = u - (R)k;
  return k;
}

struct Sep {
  double x, y, z;
};

// The tile's box, held in registers for the minimum image (block-uniform).
struct Img {
  double len[3], inv[3];
  int per[3];
  __device__ __forceinline__ explicit Img(const md_domain* D) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      len[a] = D->len[a];
      inv[a] = D->inv_len[a];
      per[a] = D->periodic[a];
    }
  }
};

// r_j - r_i under the minimum image.
__device__ __forceinline__ Sep separation(const Img& D, double4 pj, double4 pi) {
  Sep d{pj.x - pi.x, pj.y - pi.y, pj.z - pi.z};
  if (D.per[0]) d.x -= D.len[0] * rint(d.x * D.inv[0]);
  if (D.per[1]) d.y -= D.len[1] * rint(d.y * D.inv[1]);
  if (D.per[2]) d.z -= D.len[2] * rint(d.z * D.inv[2]);
  return d;
}

__device__ __forceinline__ double4 load_xyz(const double4* pos, int j) {
  // Only x, y, z: the w slot may be written concurrently by the density pass.
  const double2 a = *reinterpret_cast<const double2*>(pos + j);
  const double c = reinterpret_cast<const double*>(pos + j)[2];
  return make_double4(a.x, a.y, c, 0.0);
}

// One block: per-box sums of the tile partials in fixed order, written to
// ev[(step % ev_cap) * n_rep + rep].
__global__ __launch_bounds__(1024) void k_ev_reduce(md_batch b, const double* partial, double* ev,
                                                    int ev_cap, const md_ctl_dev* ctl) {
  __shared__ double sh[MD_EV_LEN * 16];
  const int step = ctl->step;
  double* out = ev + (size_t)(step % ev_cap) * b.n_rep * MD_EV_LEN;
  if (b.n_rep == 1) {
    double v[MD_EV_LEN];
#pragma unroll
    for (int k = 0; k < MD_EV_LEN; ++k) v[k] = 0.0;
    for (int t = threadIdx.x; t < b.n_tiles; t += blockDim.x)
#pragma unroll
      for (int k = 0; k < MD_EV_LEN; ++k) v[k] += partial[(size_t)t * MD_EV_LEN + k];
    md_block_sum<MD_EV_LEN>(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < MD_EV_LEN; ++k) out[k] = v[k];
  } else {
    const int lane = threadIdx.x & (MD_WAVE - 1), wid = threadIdx.x / MD_WAVE;
    const int nw = blockDim.x / MD_WAVE;
    for (int r = wid; r < b.n_rep; r += nw) {
      const int t0 = b.domains[r].tile_off, t1 = t0 + b.domains[r].n_tiles;
      double v[MD_EV_LEN];
#pragma unroll
      for (int k = 0; k < MD_EV_LEN; ++k) v[k] = 0.0;
      for (int t = t0 + lane; t < t1; t += MD_WAVE)
#pragma unroll
        for (int k = 0; k < MD_EV_LEN; ++k) v[k] += partial[(size_t)t * MD_EV_LEN + k];
#pragma unroll
      for (int k = 0; k < MD_EV_LEN; ++k) v[k] = md_wave_sum(v[k]);
      if (lane == 0)
#pragma unroll
        for (int k = 0; k < MD_EV_LEN; ++k) out[(size_t)r * MD_EV_LEN + k] = v[k];
    }
  }
}

// Epilogue shared by the LJ and EAM force kernels: write the force, apply the
// trailing half kick, and return the atom's kinetic energy (eV).
template <typename R>
__device__ __forceinline__ double write_force_kick(int i, int n, R fx, R fy, R fz, R* force,
                                                   double* vel, double inv_mass,
                                                   double half_dt) {
  force[i] = fx;
  force[n + i] = fy;
  force[2 * n + i] = fz;
  if (!vel) return 0.0;
  const double c = half_dt * inv_mass * MD_ACCEL;
  const double vx = vel[i] + c * (double)fx;
  const double vy = vel[n + i] + c * (double)fy;
  const double vz = vel[2 * n + i] + c * (double)fz;
  if (half_dt != 0.0) {
    vel[i] = vx;
    vel[n + i] = vy;
    vel[2 * n + i] = vz;
  }
  return 0.5 / (inv_mass * MD_ACCEL) * (vx * vx + vy * vy + vz * vz);
}

// ---------------------------------------------------------------------------
// EAM pass 1: rhobar_i = sum_j rho(r_ij), F'(rhobar_i) into pos[i].w, energy.
// ---------------------------------------------------------------------------
template <typename R, int LANES, bool EV>
__global__ __launch_bounds__(64 * LANES) void k_eam_density(
    md_batch b, double4* pos, const int* __restrict__ neigh, const int* __restrict__ nneigh,
    int npad, const R* __restrict__ rtab, const R* __restrict__ etab, TabGeom g, R rc2,
    double* saved, double* partial, md_ctl_dev* ctl) {
  constexpr int U = 4;  // neighbours in flight per lane
  __shared__ double sh[MD_EV_LEN * 16];
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;  // padding block: no block-wide work follows
  const md_tile T = b.tiles[t];
  const Img D(&b.domains[T.rep]);
  const int a = threadIdx.x / LANES, l = threadIdx.x % LANES;
  double e_acc = 0.0;
  bool oor = false;
  if (a < T.count) {
    const int i = T.first + a;
    const double4 pi = load_xyz(pos, i);
    const int nn = nneigh[i];
    const R rlo = (R)g.r_lo, rih = (R)g.r_inv_h;
    R rho = 0, phi = 0;
    const int* nb = neigh + (size_t)i * LANES + l;
    const size_t stride = (size_t)npad * LANES;
    auto pair = [&](double4 pj) {
      const Sep d = separation(D, pj, pi);
      const R x = (R)d.x, y = (R)d.y, z = (R)d.z;
      const R r2 = x * x + y * y + z * z;
      if (r2 < rc2) {
        const R r = sqrt(r2);
        R tt;
        const int k = tab_index<R>(r, rlo, rih, g.nr, tt, oor);
        const R* row = rtab + (size_t)k * MD_RTAB_W;
        rho += ((row[3] * tt + row[2]) * tt + row[1]) * tt + row[0];
        if (EV) phi += ((row[7] * tt + row[6]) * tt + row[5]) * tt + row[4];
      }
    };
    int m = l;
    for (; m + (U - 1) * LANES < nn; m += U * LANES) {
      int j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) j[u] = nb[u * stride];
      nb += U * stride;
      double4 pj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pj[u] = load_xyz(pos, j[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) pair(pj[u]);
    }
    for (; m < nn; m += LANES, nb += stride) pair(load_xyz(pos, *nb));
    rho = md_group_sum<LANES>(rho);
    if (EV) e_acc += 0.5 * (double)phi;
    if (l == 0) {
      R tt;
      const R u = (rho - (R)g.e_lo) * (R)g.e_inv_h;
      if (u < (R)0 || u > (R)g.ne) oor = true;
      const int k = tab_index<R>(rho, (R)g.e_lo, (R)g.e_inv_h, g.ne, tt, oor);
      const R* row = etab + (size_t)k * MD_ETAB_W;
      const R F = ((row[3] * tt + row[2]) * tt + row[1]) * tt + row[0];
      const R F1 = (row[6] * tt + row[5]) * tt + row[4];
      reinterpret_cast<double*>(pos + i)[3] = (double)F1;
      if (saved) {
        const int n = b.n_atoms;
        saved[i] = (double)rho;
        saved[n + i] = (double)F1;
        saved[2 * n + i] = (double)(row[8] * tt + row[7]);
      }
      if (EV) e_acc += (double)F;
    }
  }
  if (__any(oor)) {
    if ((threadIdx.x & (MD_WAVE - 1)) == 0) md_flag(ctl, MD_FLAG_TABLE_RANGE);
  }
  if (EV) {
    double v[1] = {e_acc};
    md_block_sum<1>(v, sh);
    if (threadIdx.x == 0) partial[(size_t)t * MD_EV_LEN] = v[0];
  }
}

// ---------------------------------------------------------------------------
// EAM pass 2: f_i = sum_j [phi'(r) + (F'_i + F'_j) rho'(r)] (r_j - r_i) / r,
// virial, trailing kick, kinetic energy, and the final per-box reduction.
// ---------------------------------------------------------------------------
template <typename R, int LANES, bool EV>
__global__ __launch_bounds__(64 * LANES) void k_eam_force(
    md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, const R* __restrict__ ftab, TabGeom g, R rc2,
    R* force, double* vel, double inv_mass, double half_dt, double* partial, md_ctl_dev* ctl) {
  constexpr int U = 4;  // neighbours in flight per lane
  __shared__ double sh[MD_EV_LEN * 16];
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;
  const md_tile T = b.tiles[t];
  const Img D(&b.domains[T.rep]);
  const int a = threadIdx.x / LANES, l = threadIdx.x % LANES;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // W xx yy zz xy xz yz, K
  bool oor = false;
  R fx = 0, fy = 0, fz = 0;
  R w[6] = {0, 0, 0, 0, 0, 0};
  int i = -1;
  if (a < T.count) {
    i = T.first + a;
    const double4 pi = pos[i];
    const R fpi = (R)pi.w;
    const int nn = nneigh[i];
    const R rlo = (R)g.r_lo, rih = (R)g.r_inv_h;
    const int* nb = neigh + (size_t)i * LANES + l;
    const size_t stride = (size_t)npad * LANES;
    auto pair = [&](double4 pj) {
      const Sep d = separation(D, pj, pi);
      const R x = (R)d.x, y = (R)d.y, z = (R)d.z;
      const R r2 = x * x + y * y + z * z;
      if (r2 < rc2) {
        const R rinv = rsqrt_r<R>(r2);
        const R r = r2 * rinv;
        R tt;
        const int k = tab_index<R>(r, rlo, rih, g.nr, tt, oor);
        const R* row = ftab + (size_t)k * MD_FTAB_W;
        const R dphi = (row[2] * tt + row[1]) * tt + row[0];
        const R drho = (row[5] * tt + row[4]) * tt + row[3];
        // force on i from j: s (r_j - r_i), s = [phi' + (F'_i + F'_j) rho'] / r
        const R s = (dphi + (fpi + (R)pj.w) * drho) * rinv;
        fx += s * x;
        fy += s * y;
        fz += s * z;
        if (EV) {
          w[0] -= s * x * x;
          w[1] -= s * y * y;
          w[2] -= s * z * z;
          w[3] -= s * x * y;
          w[4] -= s * x * z;
          w[5] -= s * y * z;
        }
      }
    };
    int m = l;
    for (; m + (U - 1) * LANES < nn; m += U * LANES) {
      int j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) j[u] = nb[u * stride];
      nb += U * stride;
      double4 pj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pj[u] = pos[j[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) pair(pj[u]);
    }
    for (; m < nn; m += LANES, nb += stride) pair(pos[*nb]);
  }
  fx = md_group_sum<LANES>(fx);
  fy = md_group_sum<LANES>(fy);
  fz = md_group_sum<LANES>(fz);
  if (i >= 0 && l == 0)
    acc[6] = write_force_kick<R>(i, b.n_atoms, fx, fy, fz, force, vel, inv_mass, half_dt);
  if (EV)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = 0.5 * (double)w[k];
  if (__any(oor)) {
    if ((threadIdx.x & (MD_WAVE - 1)) == 0) md_flag(ctl, MD_FLAG_TABLE_RANGE);
  }
  if (EV) {
    md_block_sum<7>(acc, sh);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 7; ++k) partial[(size_t)t * MD_EV_LEN + 1 + k] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Lennard-Jones: U = 4 eps [(s/r)^12 - (s/r)^6] - U(r_c), one pass.
// ---------------------------------------------------------------------------
struct LJc {
  double sig2, eps4, eps24, ucut;
};

template <typename R, int LANES, bool EV>
__global__ __launch_bounds__(64 * LANES) void k_lj(
    md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, LJc c, R rc2, R* force, double* vel,
    double inv_mass, double half_dt, double* partial, md_ctl_dev* ctl) {
  constexpr int U = 4;
  __shared__ double sh[MD_EV_LEN * 16];
  const int t = md_remap_block(b.n_tiles);
  if (t >= b.n_tiles) return;
  const md_tile T = b.tiles[t];
  const Img D(&b.domains[T.rep]);
  const int a = threadIdx.x / LANES, l = threadIdx.x % LANES;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // E, W xx yy zz xy xz yz, K
  const R sig2 = (R)c.sig2, eps4 = (R)c.eps4, eps24 = (R)c.eps24, ucut = (R)c.ucut;
  R fx = 0, fy = 0, fz = 0, e = 0;
  R w[6] = {0, 0, 0, 0, 0, 0};
  int i = -1;
  if (a < T.count) {
    i = T.first + a;
    const double4 pi = pos[i];
    const int nn = nneigh[i];
    const int* nb = neigh + (size_t)i * LANES + l;
    const size_t stride = (size_t)npad * LANES;
    auto pair = [&](double4 pj) {
      const Sep d = separation(D, pj, pi);
      const R x = (R)d.x, y = (R)d.y, z = (R)d.z;
      const R r2 = x * x + y * y + z * z;
      if (r2 < rc2) {
        const R ir2 = (R)1 / r2;
        const R sr2 = sig2 * ir2;
        const R sr6 = sr2 * sr2 * sr2;
        const R sr12 = sr6 * sr6;
        // f_i = -dU/dr r_ij / r = -24 eps (2 sr12 - sr6) / r^2 (r_j - r_i)
        const R s = -eps24 * ((R)2 * sr12 - sr6) * ir2;
        fx += s * x;
        fy += s * y;
        fz += s * z;
        if (EV) {
          e += eps4 * (sr12 - sr6) - ucut;
          w[0] -= s * x * x;
          w[1] -= s * y * y;
          w[2] -= s * z * z;
          w[3] -= s * x * y;
          w[4] -= s * x * z;
          w[5] -= s * y * z;
        }
      }
    };
    int m = l;
    for (; m + (U - 1) * LANES < nn; m += U * LANES) {
      int j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) j[u] = nb[u * stride];
      nb += U * stride;
      double4 pj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) pj[u] = pos[j[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) pair(pj[u]);
    }
    for (; m < nn; m += LANES, nb += stride) pair(pos[*nb]);
  }
  fx = md_group_sum<LANES>(fx);
  fy = md_group_sum<LANES>(fy);
  fz = md_group_sum<LANES>(fz);
  if (i >= 0 && l == 0)
    acc[7] = write_force_kick<R>(i, b.n_atoms, fx, fy, fz, force, vel, inv_mass, half_dt);
  if (EV) {
    acc[0] = 0.5 * (double)e;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[1 + k] = 0.5 * (double)w[k];
    md_block_sum<8>(acc, sh);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 8; ++k) partial[(size_t)t * MD_EV_LEN + k] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------
bool batch_ok(const md_batch* b) {
  return b && b->n_rep >= 1 && b->n_atoms >= 0 && b->n_tiles >= 0 && b->n_cells >= 1 &&
         b->tile_atoms == MD_TILE && b->domains && (b->tiles || b->n_tiles == 0);
}

bool nlist_ok(const md_nlist* nl) {
  if (!nl || !nl->neigh || !nl->nneigh) return false;
  const int L = nl->lanes;
  if (L != 1 && L != 2 && L != 4 && L != 8 && L != 16) return false;
  return nl->max_neigh >= L && nl->max_neigh % L == 0;
}

template <typename R, int LANES>
void launch_eam(const md_batch& b, const md_eam& p, const char* tab, const md_table_layout& TL,
                const double* pos, const md_nlist& nl, void* force, double* saved, double* vel,
                double inv_mass, double half_dt, double* ev, int ev_cap, double* partial,
                md_ctl_dev* ctl, hipStream_t st) {
  TabGeom g;
  g.r_lo = p.rho.x_lo;
  g.r_inv_h = 1.0 / p.rho.h;
  g.e_lo = p.emb.x_lo;
  g.e_inv_h = 1.0 / p.emb.h;
  g.nr = p.rho.ncoef - 3;
  g.ne = p.emb.ncoef - 3;
  const R rc2 = (R)(p.r_cut * p.r_cut);
  const dim3 grid(md_grid_blocks(b.n_tiles)), block(64 * LANES);
  const int npad = md_npad(b.n_atoms);
  const R* rtab = (const R*)(tab + TL.rtab);
  const R* ftab = (const R*)(tab + TL.ftab);
  const R* etab = (const R*)(tab + TL.etab);
  if (ev) {
    MD_LAUNCH_TIMED(MD_KERNEL_EAM_DENSITY, (k_eam_density<R, LANES, true>), grid, block, 0, st, b,
                    (double4*)pos, nl.neigh, nl.nneigh, npad, rtab, etab, g, rc2, saved, partial,
                    ctl);
    MD_LAUNCH_TIMED(MD_KERNEL_EAM_FORCE, (k_eam_force<R, LANES, true>), grid, block, 0, st, b,
                    (const double4*)pos, nl.neigh, nl.nneigh, npad, ftab, g, rc2, (R*)force, vel,
                    inv_mass, half_dt, partial, ctl);
    hipLaunchKernelGGL(k_ev_reduce, dim3(1), dim3(1024), 0, st, b, partial, ev, ev_cap, ctl);
  } else {
    MD_LAUNCH_TIMED(MD_KERNEL_EAM_DENSITY, (k_eam_density<R, LANES, false>), grid, block, 0, st,
                    b, (double4*)pos, nl.neigh, nl.nneigh, npad, rtab, etab, g, rc2, saved,
                    partial, ctl);
    MD_LAUNCH_TIMED(MD_KERNEL_EAM_FORCE, (k_eam_force<R, LANES, false>), grid, block, 0, st, b,
                    (const double4*)pos, nl.neigh, nl.nneigh, npad, ftab, g, rc2, (R*)force, vel,
                    inv_mass, half_dt, partial, ctl);
  }
}

template <typename R, int LANES>
void launch_lj(const md_batch& b, const md_lj& p, const double* pos, const md_nlist& nl,
               void* force, double* vel, double inv_mass, double half_dt, double* ev, int ev_cap,
               double* partial, md_ctl_dev* ctl, hipStream_t st) {
  LJc c;
  c.sig2 = p.sigma * p.sigma;
  c.eps4 = 4.0 * p.eps;
  c.eps24 = 24.0 * p.eps;
  const double src6 = pow(p.sigma / p.r_cut, 6.0);
  c.ucut = 4.0 * p.eps * (src6 * src6 - src6);
  const R rc2 = (R)(p.r_cut * p.r_cut);
  const dim3 grid(md_grid_blocks(b.n_tiles)), block(64 * LANES);
  const int npad = md_npad(b.n_atoms);
  if (ev) {
    MD_LAUNCH_TIMED(MD_KERNEL_LJ, (k_lj<R, LANES, true>), grid, block, 0, st, b,
                    (const double4*)pos, nl.neigh, nl.nneigh, npad, c, rc2, (R*)force, vel,
                    inv_mass, half_dt, partial, ctl);
    hipLaunchKernelGGL(k_ev_reduce, dim3(1), dim3(1024), 0, st, b, partial, ev, ev_cap, ctl);
  } else {
    MD_LAUNCH_TIMED(MD_KERNEL_LJ, (k_lj<R, LANES, false>), grid, block, 0, st, b,
                    (const double4*)pos, nl.neigh, nl.nneigh, npad, c, rc2, (R*)force, vel,
                    inv_mass, half_dt, partial, ctl);
  }
}

}  // namespace

#define MD_DISPATCH_LANES(LANES_VAR, CALL)  \
  switch (LANES_VAR) {                      \
    case 1: { constexpr int L_ = 1; CALL; } break;   \
    case 2: { constexpr int L_ = 2; CALL; } break;   \
    case 4: { constexpr int L_ = 4; CALL; } break;   \
    case 8: { constexpr int L_ = 8; CALL; } break;   \
    default: { constexpr int L_ = 16; CALL; } break; \
  }

extern "C" int md_eam_forces(const md_batch* b, const md_eam* p, md_precision prec,
                             const void* table, const double* pos, const md_nlist* nl,
                             void* force, double* saved, double* vel, double inv_mass,
                             double half_dt, double* ev, int ev_cap, void* ws, void* ctl,
                             void* stream) {
  if (!batch_ok(b) || !md_eam_ok(p) || !table || !pos || !nlist_ok(nl) || !force || !ws || !ctl)
    return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (ev && ev_cap < 1) return MD_ERR_ARG;
  if (vel && !(inv_mass > 0.0)) return MD_ERR_ARG;
  if (b->n_atoms == 0 || b->n_tiles == 0) return MD_OK;
  const md_table_layout TL = md_table_plan(p, prec);
  const md_ws_layout WL = md_ws_plan(b);
  double* partial = (double*)((char*)ws + WL.partial);
  hipStream_t st = (hipStream_t)stream;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  if (prec == MD_FP32) {
    MD_DISPATCH_LANES(nl->lanes, (launch_eam<float, L_>(*b, *p, (const char*)table, TL, pos, *nl,
                                                        force, saved, vel, inv_mass, half_dt, ev,
                                                        ev_cap, partial, c, st)));
  } else {
    MD_DISPATCH_LANES(nl->lanes, (launch_eam<double, L_>(*b, *p, (const char*)table, TL, pos, *nl,
                                                         force, saved, vel, inv_mass, half_dt, ev,
                                                         ev_cap, partial, c, st)));
  }
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" int md_lj_forces(const md_batch* b, const md_lj* p, md_precision prec,
                            const double* pos, const md_nlist* nl, void* force, double* vel,
                            double inv_mass, double half_dt, double* ev, int ev_cap, void* ws,
                            void* ctl, void* stream) {
  if (!batch_ok(b) || !p || !pos || !nlist_ok(nl) || !force || !ws || !ctl) return MD_ERR_ARG;
  if (!(p->sigma > 0.0) || !(p->r_cut > 0.0)) return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (ev && ev_cap < 1) return MD_ERR_ARG;
  if (vel && !(inv_mass > 0.0)) return MD_ERR_ARG;
  if (b->n_atoms == 0 || b->n_tiles == 0) return MD_OK;
  const md_ws_layout WL = md_ws_plan(b);
  double* partial = (double*)((char*)ws + WL.partial);
  hipStream_t st = (hipStream_t)stream;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  if (prec == MD_FP32) {
    MD_DISPATCH_LANES(nl->lanes, (launch_lj<float, L_>(*b, *p, pos, *nl, force, vel, inv_mass,
                                                       half_dt, ev, ev_cap, partial, c, st)));
  } else {
    MD_DISPATCH_LANES(nl->lanes, (launch_lj<double, L_>(*b, *p, pos, *nl, force, vel, inv_mass,
                                                        half_dt, ev, ev_cap, partial, c, st)));
  }
  MD_LAUNCH_CHECK();
  return MD_OK;
}
