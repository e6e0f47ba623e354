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

#include <mutex>
#include <type_traits>
#include <vector>

#include "md_internal.h"
#include "md_tables.h"

namespace {

template <typename R> __device__ __forceinline__ R rsqrt_r(R x);
template <> __device__ __forceinline__ double rsqrt_r<double>(double x) { return rsqrt(x); }
// v_rsq_f32 (1 ulp); squared separations are never denormal here
template <> __device__ __forceinline__ float rsqrt_r<float>(float x) { return __builtin_amdgcn_rsqf(x); }

struct TabGeom {
  double r_lo, r_inv_h, e_lo, e_inv_h;
  int nr, ne;      // intervals (FP64 r grid, embedding)
  double q_lo, q_inv_h;  // FP32 pair tables: r^2 grid of MD_STAB_N intervals
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

// Same, for a pair that may lie beyond the cutoff (masked by the caller): the
// index is clamped into the table and the range flag only counts pairs `in`.
// u = x inv_h - lo inv_h is one multiply-add.
template <typename R>
__device__ __forceinline__ int tab_index_masked(R x, R inv_h, R lo_inv_h, int nint, bool in, R& t,
                                                bool& oor) {
  const R u = x * inv_h - lo_inv_h;
  oor |= in && (u < (R)0);
  const int k = min(max((int)u, 0), nint - 1);
  t = u - (R)k;
  return k;
}

struct Sep {
  double x, y, z;
};

// The tile's box for the minimum image, in scalar registers.  The inverse length
// is 0 on non-periodic axes, where d - L rint(d * 0) = d: no selects needed.
struct Img {
  double len[3], inv[3];
  __device__ __forceinline__ explicit Img(const md_domain* D) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      len[a] = D->len[a];
      inv[a] = D->periodic[a] ? D->inv_len[a] : 0.0;
    }
  }
};

// r_j - r_i, under the minimum image when IMG (atoms whose cell stencil crosses a
// periodic boundary; for the others the plain difference is the minimum image,
// since positions are wrapped at every rebuild and drift less than half a skin).
template <bool IMG>
__device__ __forceinline__ Sep separation(const Img& D, double4 pj, double4 pi, Sep& shift) {
  Sep d{pj.x - pi.x, pj.y - pi.y, pj.z - pi.z};
  if (IMG) {
    shift.x = D.len[0] * rint(d.x * D.inv[0]);
    shift.y = D.len[1] * rint(d.y * D.inv[1]);
    shift.z = D.len[2] * rint(d.z * D.inv[2]);
    d.x -= shift.x;
    d.y -= shift.y;
    d.z -= shift.z;
  }
  return d;
}

// Rows of the pair tables: the r grid's intervals (FP64), the r^2 grid's and its zero
// row (FP32).
template <typename R>
__device__ __host__ __forceinline__ int pair_rows(const TabGeom& g) {
  return sizeof(R) == 4 ? MD_STAB_ROWS : g.nr;
}

// FP32 pair-table row and local coordinate for squared distance q (r^2 grid).  Every q
// at or beyond r_cut^2 lands on the zero row MD_STAB_N, so such pairs add exactly zero
// with no compare; q below the table clamps to row 0 (flagged by the density pass).
// t = fract(u) equals u - floor(u) exactly for u >= 0.
__device__ __forceinline__ int qtab_index(float q, float inv_h, float lo_inv_h, float& t) {
  const float u = q * inv_h - lo_inv_h;
  t = __builtin_amdgcn_fractf(u);
  return min(max((int)u, 0), MD_STAB_N);
}

__device__ __forceinline__ float cubic(const float* a, float t) {
  return ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
}

// Blocks of the force passes: up to 1024 threads (md_nlist.block: 256, 512 or 1024, default
// 1024), each block TPB work tiles of 64 atoms x LANES lanes.
constexpr int FBLOCK = 1024;
template <int LANES>
__device__ __forceinline__ int tiles_per_block() {
  return __builtin_amdgcn_readfirstlane((int)blockDim.x / (64 * LANES));
}
static inline int block_threads(const md_nlist& nl) { return nl.block ? nl.block : FBLOCK; }

// Where a thread sits: its tile (-1 if none), its atom slot and lane.
struct Slot {
  int t, a, l;
};
template <int LANES>
__device__ __forceinline__ Slot force_slot(int n_tiles) {
  const int TPB = tiles_per_block<LANES>();
  const int nlb = (n_tiles + TPB - 1) / TPB;
  const int lb = md_remap_block(nlb);
  Slot s;
  const int within = threadIdx.x % (64 * LANES);
  // a tile spans whole wavefronts, so the tile index is wave-uniform (scalar registers)
  s.t = __builtin_amdgcn_readfirstlane(lb * TPB + (int)threadIdx.x / (64 * LANES));
  if (lb >= nlb || s.t >= n_tiles) s.t = -1;
  s.a = within / LANES;
  s.l = within % LANES;
  return s;
}

// Stage a table of nrows rows of W values of type R into LDS (16-byte moves).
template <typename R, int W>
__device__ __forceinline__ const R* stage_table(const R* g, int nrows, R* lds) {
  const int n16 = nrows * W * (int)sizeof(R) / 16;
  const float4* src = reinterpret_cast<const float4*>(g);
  float4* dst = reinterpret_cast<float4*>(lds);
  for (int q = threadIdx.x; q < n16; q += blockDim.x) dst[q] = src[q];
  __syncthreads();
  return lds;
}

// Gathers address a uniform base plus a 32-bit byte offset (one VALU op per
// address; arrays are below 4 GiB).
__device__ __forceinline__ double4 load_xyz(const double4* pos, int j) {
  // Only x, y, z: the w slot may be written concurrently by the density pass.
  const char* p = reinterpret_cast<const char*>(pos) + (uint32_t)((uint32_t)j << 5);
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double c = *reinterpret_cast<const double*>(p + 16);
  return make_double4(a.x, a.y, c, 0.0);
}

__device__ __forceinline__ double4 load_rec(const double4* pos, int j) {
  return *reinterpret_cast<const double4*>(reinterpret_cast<const char*>(pos) +
                                           (uint32_t)((uint32_t)j << 5));
}

// Neighbour records of the FP32 force pass: 16 bytes {u_x, u_y, u_z, F'} with the
// coordinates in fixed point, u = rint((x - lo) 2^32 / span) mod 2^32 per axis.  On a
// periodic axis span = L, so the wrapped 32-bit difference of two coordinates is the
// minimum image (no branch, no rounding per pair); on other axes span = max(L, 4 r_ns),
// and listed pairs (|d| < r_ns < span / 2) never alias, wherever the atoms are.  One
// 16-byte load per neighbour instead of two for the FP64 record.
struct FixBox {
  double lo[3], scale[3];  // 2^32 / span
  float inv[3];            // span / 2^32
  bool iso;                // one span on all axes
};
// The scale 2^32 / span comes from the domain's stored 1 / L wherever span = L (so that
// L scale = 2^32 to 1e-16 and an image shift of L is 2^32 fixed-point units); a division
// is left only for short non-periodic axes.
__device__ __forceinline__ FixBox fix_box(const md_domain& D, double r_ns) {
  FixBox f;
  double span[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const bool full = D.periodic[a] || D.len[a] >= 4.0 * r_ns;
    span[a] = full ? D.len[a] : 4.0 * r_ns;
    f.lo[a] = D.lo[a];
    f.scale[a] = full ? 4294967296.0 * D.inv_len[a] : 4294967296.0 / span[a];
    f.inv[a] = (float)(span[a] * 2.3283064365386963e-10);
  }
  f.iso = span[0] == span[1] && span[0] == span[2];
  return f;
}

__device__ __forceinline__ uint32_t fix_coord(double x, double lo, double scale) {
  const double r = rint((x - lo) * scale);
  const double q = floor(r * 2.3283064365386963e-10);  // r = q 2^32 + (r mod 2^32), exact
  return (uint32_t)(r - q * 4294967296.0);
}
// Separation r_j - r_i of two fixed-point records: in angstrom, or (ISO: all axes share
// one scale) in fixed-point steps, the scale then folded into the caller's table
// coordinate and force factor, three multiplies fewer per pair.
template <bool ISO>
__device__ __forceinline__ void fix_sep(const uint4& q, const uint4& ri, const FixBox& X,
                                        float& x, float& y, float& z) {
  x = (float)(int)(q.x - ri.x);
  y = (float)(int)(q.y - ri.y);
  z = (float)(int)(q.z - ri.z);
  if (!ISO) {
    x *= X.inv[0];
    y *= X.inv[1];
    z *= X.inv[2];
  }
}

// Fixed-point coordinates of the atoms of a batch (the x, y, z words of the FP32 neighbour
// records of the LJ and EAM passes; the EAM density pass adds F' in the w word).
// ctl: not NULL when the records were carried over from the last force pass (md_drift.rec_in):
// they are then remade only if positions changed since by anything else (ctl->rec_stale).
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_fix_records(md_batch b, const double4* pos,
                                                                uint4* rec,
                                                                const md_ctl_dev* ctl) {
  if (ctl && !ctl->rec_stale) return;
  const int nlb = (b.n_tiles + 3) / 4;
  const int lane = threadIdx.x & (MD_WAVE - 1);
  for (int k = 0;; ++k) {
    const int lb = md_remap_stride(nlb, k);
    if (lb >= nlb) break;
    const int tile = lb * 4 + (int)(threadIdx.x / MD_WAVE);
    if (tile >= b.n_tiles) continue;
    const md_tile T = b.tiles[tile];
    if (lane >= T.count) continue;
    const int i = T.first + lane;
    const FixBox X = fix_box(b.domains[T.rep], b.r_ns);
    const double2 xy = *reinterpret_cast<const double2*>(pos + i);
    const double z = reinterpret_cast<const double*>(pos + i)[2];
    rec[i] = make_uint4(fix_coord(xy.x, X.lo[0], X.scale[0]), fix_coord(xy.y, X.lo[1], X.scale[1]),
                        fix_coord(z, X.lo[2], X.scale[2]), 0u);
  }
}
__device__ __forceinline__ uint4 load_rec16(const uint4* rec, int j) {
  return *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(rec) +
                                         (uint32_t)((uint32_t)j << 4));
}

// List entries are addressed with 32-bit byte offsets when the list holds fewer
// than 2^30 entries (E = uint32_t), with 64-bit element offsets otherwise.
__device__ __forceinline__ int load_idx(const int* neigh, uint32_t e) {
  return *reinterpret_cast<const int*>(reinterpret_cast<const char*>(neigh) + (e << 2));
}
__device__ __forceinline__ int load_idx(const int* neigh, uint64_t e) { return neigh[e]; }

// Visit the nn list entries of one atom handled by lane l of LANES: entry m sits
// at element ((m / LANES) * npad + i) * LANES + l, i.e. e0 + (m / LANES) * stride.
// U entries are in flight per lane: indices first, then records, then the math.
template <int LANES, int U, typename E, typename Load, typename Pair>
__device__ __forceinline__ void visit_list(const int* neigh, E e0, E stride, int l, int nn,
                                           Load load, Pair pair) {
  int m = l;
  E e = e0;
  for (; m + (U - 1) * LANES < nn; m += U * LANES) {
    int j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = load_idx(neigh, e + u * stride);
    e += U * stride;
    decltype(load(0)) q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = load(j[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) pair(q[u]);
  }
  for (; m < nn; m += LANES, e += stride) pair(load(load_idx(neigh, e)));
}

// Software-pipelined variant for the EAM passes: the list indices of the next U
// entries are loaded while the records of the current U are in flight, so a lane
// waits for one round trip per U entries instead of two.  All loads are issued
// unconditionally in a fixed order (entries past the lane's end read the atom's
// first entry and are replaced by the atom itself, `self`), so the compiler can
// wait for the records alone; pair(q, valid) masks the padding.
template <int LANES, int U, typename E, typename Load, typename Pair>
__device__ __forceinline__ void visit_list_pipe(const int* neigh, E e0, E stride, int l, int nn,
                                                int self, Load load, Pair pair) {
  const int cnt = nn > l ? (nn - l + LANES - 1) / LANES : 0;  // this lane's entries
  int jn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) jn[u] = load_idx(neigh, u < cnt ? e0 + u * stride : e0);
  E e = e0 + U * stride;
  for (int b0 = 0; b0 < cnt; b0 += U) {
    decltype(load(0)) q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = load(b0 + u < cnt ? jn[u] : self);
#pragma unroll
    for (int u = 0; u < U; ++u) jn[u] = load_idx(neigh, b0 + U + u < cnt ? e + u * stride : e0);
    e += U * stride;
#pragma unroll
    for (int u = 0; u < U; ++u) pair(q[u], b0 + u < cnt);
  }
}

// F'(rhobar) travels to the force pass in the w slot of the position record: as a
// double in FP64, as the float in its low word in FP32 (no conversion per pair).
template <typename R> __device__ __forceinline__ void store_fp(double4* pos, int i, R v);
template <> __device__ __forceinline__ void store_fp<double>(double4* pos, int i, double v) {
  reinterpret_cast<double*>(pos + i)[3] = v;
}
template <> __device__ __forceinline__ void store_fp<float>(double4* pos, int i, float v) {
  reinterpret_cast<double*>(pos + i)[3] = __hiloint2double(0, __float_as_int(v));
}
template <typename R> __device__ __forceinline__ R load_fp(double w);
template <> __device__ __forceinline__ double load_fp<double>(double w) { return w; }
template <> __device__ __forceinline__ float load_fp<float>(double w) {
  return __int_as_float(__double2loint(w));
}

template <typename R> __device__ __forceinline__ R sqrt_r(R x);
template <> __device__ __forceinline__ double sqrt_r<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float sqrt_r<float>(float x) {
  return x * __builtin_amdgcn_rsqf(x);
}

// Per-box records are 64-bit fixed point (MD_EV_SCALE units per eV): integer
// additions are associative, so atomically accumulated records are bit-for-bit
// reproducible whatever order the blocks finish in.
__device__ __forceinline__ long long to_fixed(double v) {
  return (long long)rint(v * MD_EV_SCALE);
}

// Add a block's per-tile sums (tsum[g][k], g < TPB) into the record slot: tiles
// of one box are combined first, then one atomic per (box, component).
__device__ __forceinline__ void accumulate_record(const md_batch& b, int TPB, int lb, int nlb,
                                                  const double* tsum, long long* slot) {
  const int k = threadIdx.x;
  if (k >= MD_EV_LEN || lb >= nlb) return;
  int rep = -1;
  double acc = 0.0;
  for (int g = 0; g < TPB; ++g) {
    const int t = lb * TPB + g;
    if (t >= b.n_tiles) break;
    const int r = b.tiles[t].rep;
    if (r != rep) {
      if (rep >= 0) atomicAdd((unsigned long long*)&slot[(size_t)rep * MD_EV_LEN + k],
                              (unsigned long long)to_fixed(acc));
      rep = r;
      acc = 0.0;
    }
    acc += tsum[g * MD_EV_LEN + k];
  }
  if (rep >= 0)
    atomicAdd((unsigned long long*)&slot[(size_t)rep * MD_EV_LEN + k],
              (unsigned long long)to_fixed(acc));
}

// Zero the record slot of the current step (one block, before any accumulation).
__device__ __forceinline__ void zero_record(const md_batch& b, long long* ev, int ev_cap,
                                            int step) {
  long long* slot = ev + (size_t)(step % ev_cap) * b.n_rep * MD_EV_LEN;
  for (int q = threadIdx.x; q < b.n_rep * MD_EV_LEN; q += blockDim.x) slot[q] = 0;
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
  const double vx = md_kick(vel[i], c, (double)fx);
  const double vy = md_kick(vel[n + i], c, (double)fy);
  const double vz = md_kick(vel[2 * n + i], c, (double)fz);
  if (half_dt != 0.0) {
    vel[i] = vx;
    vel[n + i] = vy;
    vel[2 * n + i] = vz;
  }
  return 0.5 / (inv_mass * MD_ACCEL) * md_norm2(vx, vy, vz);
}


// ---------------------------------------------------------------------------
// EAM pass 1: rhobar_i = sum_j rho(r_ij), F'(rhobar_i) into pos[i].w, energy.
// ---------------------------------------------------------------------------
template <typename R, int LANES, bool EV, bool TLDS, int U, typename E>
__device__ __forceinline__ void eam_density_body(
    const md_batch& b, double4* pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, const R* __restrict__ rtab_g,
    const R* __restrict__ etab, const TabGeom& g, R rc2, double* saved, double* partial,
    uint4* rec, long long* ev, int ev_cap, int rec_verify, md_ctl_dev* ctl) {
  extern __shared__ float4 s_dyn[];
  __shared__ double sh[MD_EV_LEN * 16];
  const R* rtab = TLDS ? stage_table<R, MD_RTAB_W>(rtab_g, pair_rows<R>(g), (R*)s_dyn) : rtab_g;
  if (EV && blockIdx.x == 0) zero_record(b, ev, ev_cap, ctl->step_next);
  md_step_bookkeeping(ctl, rec_verify != 0);
  const Slot S = force_slot<LANES>(b.n_tiles);
  double e_acc = 0.0;
  bool oor = false;
  int i = -1, nn = 0, raw = 0;
  md_tile T{0, 0, 0, 0};
  if (S.t >= 0) {
    T = b.tiles[S.t];
    if (S.a < T.count) {
      i = T.first + S.a;
      raw = nneigh[i];
      nn = raw & MD_NN_MASK;
    }
  }
  const bool wimg = __any(raw & MD_NN_IMG);
  R rho = 0, phi = 0;
  float min_r2 = 3.0e38f;  // FP32: smallest r^2 seen (range check against the table)
  double min_r2_scale = 1.0;
  if constexpr (std::is_same<R, float>::value) {
    if (i >= 0) {
      // separations from the fixed-point records of k_fix_records (as in the force pass)
      const FixBox X = fix_box(b.domains[T.rep], b.r_ns);
      const uint4 ri = rec[i];
      const double s = X.inv[0];
      const E e0 = (E)i * LANES + S.l, stride = (E)npad * LANES;
      auto run32 = [&](auto iso_tag) {
        constexpr bool ISO = decltype(iso_tag)::value;
        const float qih = (float)(ISO ? g.q_inv_h * s * s : g.q_inv_h);
        const float qloh = (float)(g.q_lo * g.q_inv_h);
        auto pair = [&](uint4 q, bool valid) {
          float x, y, z;
          fix_sep<ISO>(q, ri, X, x, y, z);
          // padding entries (the atom itself) are moved beyond the cutoff
          const float r2 = valid ? x * x + y * y + z * z : 1e30f;
          // r^2 table: no square root; pairs beyond r_c read the zero row, below the
          // table shows in the smallest r^2
          float tt;
          const float* row = rtab + qtab_index(r2, qih, qloh, tt) * MD_RTAB_W;
          min_r2 = fminf(min_r2, r2);
          rho += cubic(row, tt);
          if (EV) phi += cubic(row + 4, tt);
        };
        visit_list_pipe<LANES, U>(neigh, e0, stride, S.l, nn, i,
                                  [&](int j) { return load_rec16(rec, j); }, pair);
      };
      if (X.iso) {
        run32(std::true_type{});
        min_r2_scale = s * s;
      } else {
        run32(std::false_type{});
      }
    }
  } else if (i >= 0) {
    const Img D(&b.domains[T.rep]);
    const double4 pi = load_xyz(pos, i);
    const R rih = (R)g.r_inv_h, rloh = (R)(g.r_lo * g.r_inv_h);
    const E e0 = (E)i * LANES + S.l, stride = (E)npad * LANES;
    auto run = [&](auto img_tag) {
      constexpr bool IMG = decltype(img_tag)::value;
      auto pair = [&](double4 pj, bool valid) {
        Sep sh;
        const Sep d = separation<IMG>(D, pj, pi, sh);
        const R x = (R)d.x, y = (R)d.y, z = (R)d.z;
        // padding entries (the atom itself) are moved out of range
        const R r2 = valid ? x * x + y * y + z * z : (R)1e30;
        const bool in = r2 < rc2;  // branch-free: pairs beyond r_c are masked
        const R r = sqrt_r<R>(r2);
        R tt;
        const int k = tab_index_masked<R>(r, rih, rloh, g.nr, in, tt, oor);
        const R* row = rtab + k * MD_RTAB_W;
        const R vr = ((row[3] * tt + row[2]) * tt + row[1]) * tt + row[0];
        const R vp = EV ? ((row[7] * tt + row[6]) * tt + row[5]) * tt + row[4] : (R)0;
        rho += in ? vr : (R)0;
        if (EV) phi += in ? vp : (R)0;
      };
      visit_list_pipe<LANES, U>(neigh, e0, stride, S.l, nn, i,
                                [&](int j) { return load_xyz(pos, j); }, pair);
    };
    if (wimg) run(std::true_type{});
    else run(std::false_type{});
  }
  if (std::is_same<R, float>::value && (double)min_r2 * min_r2_scale < g.q_lo) oor = true;
  rho = md_group_sum<LANES>(rho);
  if (i >= 0) {
    if (EV) e_acc += 0.5 * (double)phi;
    if (S.l == 0) {
      R tt;
      const R u = (rho - (R)g.e_lo) * (R)g.e_inv_h;
      if (u < (R)0 || u > (R)g.ne) oor = true;
      const int k = tab_index<R>(rho, (R)g.e_lo, (R)g.e_inv_h, g.ne, tt, oor);
      const R* row = etab + (size_t)k * MD_ETAB_W;
      const R F = ((row[3] * tt + row[2]) * tt + row[1]) * tt + row[0];
      const R F1 = (row[6] * tt + row[5]) * tt + row[4];
      store_fp<R>(pos, i, F1);
      // F' completes the atom's record for the force pass (other blocks read only its
      // x, y, z words in this pass)
      if (rec) reinterpret_cast<uint32_t*>(rec + i)[3] = __float_as_uint((float)F1);
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
    double res;
    int gg, kk;
    if (md_group_waves_sum<1>(v, LANES, sh, res, gg, kk)) {
      const int TPB = tiles_per_block<LANES>();
      const int nlb = (b.n_tiles + TPB - 1) / TPB;
      const int lb = md_remap_block(nlb);
      const int t = lb * TPB + gg;
      if (lb < nlb && t < b.n_tiles) partial[(size_t)t * MD_EV_LEN] = res;
    }
  }
}

// One density kernel per precision (their register budgets differ).  FP32 keeps 8
// neighbours in flight per lane.
#define MD_EAM_DENSITY_ARGS(R)                                                                 \
  md_batch b, double4 *pos, const int *__restrict__ neigh, const int *__restrict__ nneigh,   \
      int npad, const R *__restrict__ rtab_g, const R *__restrict__ etab, TabGeom g, R rc2,  \
      double *saved, double *partial, uint4 *rec, long long *ev, int ev_cap, int rec_verify,    \
      md_ctl_dev *ctl
template <int LANES, bool EV, bool TLDS, typename E>
__global__ __launch_bounds__(FBLOCK) void k_eam_density_f32(MD_EAM_DENSITY_ARGS(float)) {
  eam_density_body<float, LANES, EV, TLDS, 8, E>(b, pos, neigh, nneigh, npad, rtab_g, etab, g, rc2,
                                           saved, partial, rec, ev, ev_cap, rec_verify, ctl);
}
template <int LANES, bool EV, bool TLDS, typename E>
__global__ __launch_bounds__(FBLOCK) void k_eam_density_f64(MD_EAM_DENSITY_ARGS(double)) {
  eam_density_body<double, LANES, EV, TLDS, 4, E>(b, pos, neigh, nneigh, npad, rtab_g, etab, g, rc2,
                                            saved, partial, nullptr, ev, ev_cap, rec_verify, ctl);
}
#undef MD_EAM_DENSITY_ARGS

// Density pass for fixed positions whose density Jacobian jac[i][k] = d rhobar_i /
// d c_rho_k is kept: rhobar_i = sum_k c_rho_k jac[i][k].  Each wavefront takes 64
// consecutive atoms, eight at a time: a group of 16 lanes reads one atom's row (lane q
// entries q, q + 16, ...: one cache line per group and load; all NJ = ceil(n_rho / 16)
// loads of two atoms issued together, entries past the row clamped to its last one with
// a zero coefficient) and adds it up by a group butterfly; then the embedding as in the
// pair-loop pass with one atom per lane.
template <typename R, int NJ>
__global__ __launch_bounds__(MD_ATOM_BLOCK) void k_eam_density_jac(
    int n, double4* pos, const double* __restrict__ jac, const double* __restrict__ c_rho,
    int n_rho, const R* __restrict__ etab, TabGeom g, double* saved, uint4* rec,
    md_ctl_dev* ctl) {
  __shared__ double s_rho[MD_ATOM_BLOCK];
  const int lane = threadIdx.x & (MD_WAVE - 1);
  double* wrho = s_rho + (threadIdx.x - lane);  // this wavefront's 64 sums
  const int a0 = ((blockIdx.x * blockDim.x + threadIdx.x) / MD_WAVE) * MD_WAVE;
  if (a0 >= n) return;  // whole wavefronts
  const int na = min(MD_WAVE, n - a0);
  const int grp = lane >> 4, q = lane & 15;
  double c[NJ];
  int kk[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int k = q + 16 * j;
    c[j] = k < n_rho ? c_rho[k] : 0.0;
    kk[j] = k < n_rho ? k : n_rho - 1;
  }
  for (int a = grp; a < na; a += 8) {
    const int b2 = a + 4 < na ? a + 4 : a;  // the second atom (or the first again)
    const double* r0 = jac + (size_t)(a0 + a) * n_rho;
    const double* r1 = jac + (size_t)(a0 + b2) * n_rho;
    double x0[NJ], x1[NJ];
    // streamed once per pass: kept out of the way of the force pass's cached records
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      x0[j] = __builtin_nontemporal_load(r0 + kk[j]);
      x1[j] = __builtin_nontemporal_load(r1 + kk[j]);
    }
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      v0 = fma(c[j], x0[j], v0);
      v1 = fma(c[j], x1[j], v1);
    }
    v0 = md_group_sum<16>(v0);
    v1 = md_group_sum<16>(v1);
    if (q == 0) {
      wrho[a] = v0;
      wrho[b2] = v1;  // b2 == a: the same value again
    }
  }
  __builtin_amdgcn_wave_barrier();
  const double mine = lane < na ? wrho[lane] : 0.0;
  bool oor = false;
  if (lane < na) {
    const int i = a0 + lane;
    const R rho = (R)mine;
    R tt;
    const R u = (rho - (R)g.e_lo) * (R)g.e_inv_h;
    if (u < (R)0 || u > (R)g.ne) oor = true;
    const int k = tab_index<R>(rho, (R)g.e_lo, (R)g.e_inv_h, g.ne, tt, oor);
    const R* row = etab + (size_t)k * MD_ETAB_W;
    const R F1 = (row[6] * tt + row[5]) * tt + row[4];
    store_fp<R>(pos, i, F1);
    if (rec) reinterpret_cast<uint32_t*>(rec + i)[3] = __float_as_uint((float)F1);
    if (saved) {
      saved[i] = (double)rho;
      saved[n + i] = (double)F1;
      saved[2 * n + i] = (double)(row[8] * tt + row[7]);
    }
  }
  if (__any(oor)) {
    if (lane == 0) md_flag(ctl, MD_FLAG_TABLE_RANGE);
  }
}

// ---------------------------------------------------------------------------
// EAM pass 2: f_i = sum_j [phi'(r) + (F'_i + F'_j) rho'(r)] (r_j - r_i) / r,
// virial, trailing kick and kinetic energy.
// ---------------------------------------------------------------------------
// The next step's kick-drift fused into the force pass (md_drift): new positions
// go to pos_out (pos is still being read by other blocks), velocities advance to
// the half step, and the block's displacement maximum is published.
struct DriftArgs {
  double4* pos_out;  // nullptr: no fused drift
  const double* pos_ref;
  double dt, thr2;
  md_walls_dev w;
  uint4* rec_in;   // FP32 records of pos carried over from the last force pass, or nullptr
  uint4* rec_out;  // FP32 records of pos_out written by the fused drift, or nullptr
  int rec_current; // rec_in declared current: no records kernel, verified on the device
  md_langevin_dev L;  // the Langevin update before the next half kick (L.n = 0: none)
};

// Epilogue of a force pass with the next kick-drift fused in: write the force, apply
// the trailing half kick of this step (its kinetic energy is returned), then the next
// step's Langevin update (NVT) if any, half kick and drift with the walls at (step + 1) dt
// -- the same operations, in the same order, as md_verlet_step(MD_KICK_DRIFT) -- into
// dr.pos_out; d2max gets the
// atom's displacement from x_ref.  In FP32 with dr.rec_out, the new position's fixed-point
// record (as k_fix_records would make it, in the atom's box D) goes there too.
template <typename R, bool THERMO>
__device__ __forceinline__ double fused_kick_drift(int i, int n, R fx, R fy, R fz, R* force,
                                                   double* vel, double inv_mass, double half_dt,
                                                   const double4* pos, const DriftArgs& dr,
                                                   int step, const md_domain& D, double r_ns,
                                                   double& d2max, int& bad) {
  force[i] = fx;
  force[n + i] = fy;
  force[2 * n + i] = fz;
  const double c = half_dt * inv_mass * MD_ACCEL;
  const double F[3] = {(double)fx, (double)fy, (double)fz};
  double v[3] = {md_kick(vel[i], c, F[0]), md_kick(vel[n + i], c, F[1]),
                  md_kick(vel[2 * n + i], c, F[2])};
  const double ke = 0.5 / (inv_mass * MD_ACCEL) * md_norm2(v[0], v[1], v[2]);
  const double4 p = pos[i];
  double x[3] = {p.x, p.y, p.z};
  if (THERMO) md_langevin_atom(dr.L, D, i, step + 1, x, v);
  v[0] = md_kick(v[0], c, F[0]);
  v[1] = md_kick(v[1], c, F[1]);
  v[2] = md_kick(v[2], c, F[2]);
  md_drift_atom(x, v, dr.dt, dr.w, (double)(step + 1) * dr.dt);
  vel[i] = v[0];
  vel[n + i] = v[1];
  vel[2 * n + i] = v[2];
  dr.pos_out[i] = make_double4(x[0], x[1], x[2], p.w);
  if (std::is_same<R, float>::value && dr.rec_out) {
    const FixBox X = fix_box(D, r_ns);
    dr.rec_out[i] = make_uint4(fix_coord(x[0], X.lo[0], X.scale[0]),
                               fix_coord(x[1], X.lo[1], X.scale[1]),
                               fix_coord(x[2], X.lo[2], X.scale[2]), 0u);
  }
  if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2])) bad |= MD_FLAG_NONFINITE;
  d2max = md_disp2(x, dr.pos_ref, i, n);
  return ke;
}

template <typename R, int LANES, bool EV, bool TLDS, typename E, bool THERMO>
__device__ __forceinline__ void eam_force_body(
    const md_batch& b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, const R* __restrict__ ftab_g, const TabGeom& g,
    R rc2, R* force, double* vel, double inv_mass, double half_dt, const DriftArgs& dr,
    const double* partial, const uint4* rec, long long* ev, int ev_cap, md_ctl_dev* ctl) {
  constexpr bool FP32 = std::is_same<R, float>::value;
  constexpr int U = 4;  // (8 in flight measured slower here: the gathers contend)
  extern __shared__ float4 s_dyn[];
  __shared__ double sh[MD_EV_LEN * 16];
  __shared__ double tsum[MD_EV_LEN * 16];
  const R* ftab = TLDS ? stage_table<R, MD_FTAB_W>(ftab_g, pair_rows<R>(g), (R*)s_dyn) : ftab_g;
  const Slot S = force_slot<LANES>(b.n_tiles);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // W xx yy zz xy xz yz, K
  R fx = 0, fy = 0, fz = 0;
  R w[6] = {0, 0, 0, 0, 0, 0};
  int i = -1, nn = 0, raw = 0;
  md_tile T{0, 0, 0, 0};
  if (S.t >= 0) {
    T = b.tiles[S.t];
    if (S.a < T.count) {
      i = T.first + S.a;
      raw = nneigh[i];
      nn = raw & MD_NN_MASK;
    }
  }
  const bool wimg = __any(raw & MD_NN_IMG);
  if constexpr (FP32) {
    if (i >= 0) {
      // separations from the fixed-point records (the minimum image by 32-bit wrap-around);
      // the virial is accumulated per pair, W = 1/2 sum_ij r_ij (x) f_ij.  (Folding a
      // common scale into the table coordinate, as the density pass does, measured slower
      // here: 27.0 against 25.9 us on 131k Cu.)
      const FixBox X = fix_box(b.domains[T.rep], b.r_ns);
      const uint4 ri = rec[i];
      const float fpi = __uint_as_float(ri.w);
      const float qih = (float)g.q_inv_h, qloh = (float)(g.q_lo * g.q_inv_h);
      const E e0 = (E)i * LANES + S.l, stride = (E)npad * LANES;
      auto pair = [&](uint4 q, bool) {
        float x, y, z;
        fix_sep<false>(q, ri, X, x, y, z);
        const float r2 = x * x + y * y + z * z;
        // s = [phi'(r) + (F'_i + F'_j) rho'(r)] / r; the force on i from j is s (r_j - r_i).
        // Pairs beyond r_c read the zero row (s = 0); a padding entry is the atom itself, at
        // zero separation, so it adds nothing either.
        float tt;
        const float* row = ftab + qtab_index(r2, qih, qloh, tt) * MD_FTAB_W;
        const float sv = cubic(row, tt) + (fpi + __uint_as_float(q.w)) * cubic(row + 4, tt);
        const float px = sv * x, py = sv * y, pz = sv * z;
        fx += px;
        fy += py;
        fz += pz;
        if (EV) {  // r_ij (x) f_ij with r_ij = -(x, y, z)
          w[0] -= x * px;
          w[1] -= y * py;
          w[2] -= z * pz;
          w[3] -= x * py;
          w[4] -= x * pz;
          w[5] -= y * pz;
        }
      };
      visit_list_pipe<LANES, U>(neigh, e0, stride, S.l, nn, i,
                                [&](int j) { return load_rec16(rec, j); }, pair);
    }
  } else if (i >= 0) {
    const Img D(&b.domains[T.rep]);
    const double4 pi = pos[i];
    const R fpi = load_fp<R>(pi.w);
    const R rih = (R)g.r_inv_h, rloh = (R)(g.r_lo * g.r_inv_h);
    const E e0 = (E)i * LANES + S.l, stride = (E)npad * LANES;
    auto run = [&](auto img_tag) {
      constexpr bool IMG = decltype(img_tag)::value;
      auto pair = [&](double4 pj, bool valid) {
        Sep sh;
        const Sep d = separation<IMG>(D, pj, pi, sh);
        const R x = (R)d.x, y = (R)d.y, z = (R)d.z;
        const R r2 = x * x + y * y + z * z;
        const bool in = valid && r2 < rc2;  // branch-free: pairs beyond r_c are masked
        // s = [phi'(r) + (F'_i + F'_j) rho'(r)] / r; the force on i from j is s (r_j - r_i).
        // (Pairs below the table are flagged by the density pass, which sees the same r.)
        const R rinv = rsqrt_r<R>(r2);
        const R r = r2 * rinv;
        R tt;
        bool below = false;
        const int k = tab_index_masked<R>(r, rih, rloh, g.nr, in, tt, below);
        const R* row = ftab + k * MD_FTAB_W;
        const R dphi = (row[2] * tt + row[1]) * tt + row[0];
        const R drho = (row[5] * tt + row[4]) * tt + row[3];
        const R s0 = (dphi + (fpi + load_fp<R>(pj.w)) * drho) * rinv;
        const R s = in ? s0 : (R)0;
        const R px = s * x, py = s * y, pz = s * z;
        fx += px;
        fy += py;
        fz += pz;
        if (EV && IMG) {
          // virial: W = sum_i x_i (x) F_i + 1/2 sum_ij c_ij (x) f_ij, c_ij the image
          // shift of the pair (zero for pairs that do not cross the boundary)
          const R cx = (R)sh.x, cy = (R)sh.y, cz = (R)sh.z;
          w[0] += cx * px;
          w[1] += cy * py;
          w[2] += cz * pz;
          w[3] += cx * py;
          w[4] += cx * pz;
          w[5] += cy * pz;
        }
      };
      visit_list_pipe<LANES, U>(neigh, e0, stride, S.l, nn, i,
                                [&](int j) { return load_rec(pos, j); }, pair);
    };
    if (wimg) run(std::true_type{});
    else run(std::false_type{});
  }
  fx = md_group_sum<LANES>(fx);
  fy = md_group_sum<LANES>(fy);
  fz = md_group_sum<LANES>(fz);
  if (EV)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = 0.5 * (double)w[k];
  double d2max = 0.0;
  int bad = 0;
  if (i >= 0 && S.l == 0) {
    if (dr.pos_out) {
      acc[6] = fused_kick_drift<R, THERMO>(i, b.n_atoms, fx, fy, fz, force, vel, inv_mass,
                                           half_dt, pos,
                                   dr, ctl->step, b.domains[T.rep], b.r_ns, d2max, bad);
    } else {
      acc[6] = write_force_kick<R>(i, b.n_atoms, fx, fy, fz, force, vel, inv_mass, half_dt);
    }
    if (EV && !FP32) {
      // x_i (x) F_i: the atom's position with its total force (FP64)
      const double4 pi = load_xyz(pos, i);
      const double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
      acc[0] += pi.x * Fx;
      acc[1] += pi.y * Fy;
      acc[2] += pi.z * Fz;
      acc[3] += pi.x * Fy;
      acc[4] += pi.x * Fz;
      acc[5] += pi.y * Fz;
    }
  }
  if (EV) {
    double res;
    int gg, kk;
    const int TPB = tiles_per_block<LANES>();
    const int nlb = (b.n_tiles + TPB - 1) / TPB;
    const int lb = md_remap_block(nlb);
    if (md_group_waves_sum<7>(acc, LANES, sh, res, gg, kk)) {
      tsum[gg * MD_EV_LEN + 1 + kk] = res;
      const int t = lb * TPB + gg;
      // the tile's energy from the density pass
      if (kk == 0) tsum[gg * MD_EV_LEN] = (lb < nlb && t < b.n_tiles) ? partial[(size_t)t * MD_EV_LEN] : 0.0;
    }
    __syncthreads();
    accumulate_record(b, TPB, lb, nlb, tsum, ev + (size_t)(ctl->step % ev_cap) * b.n_rep * MD_EV_LEN);
  }
  // positions move without new records: carried records are void from here on
  if (dr.pos_out && !dr.rec_out && blockIdx.x == 0 && threadIdx.x == 0) ctl->rec_stale = 1;
  if (dr.pos_out) md_publish_dmax(d2max, bad, dr.thr2, ctl);
}

// One kernel per precision (their register budgets differ).  Holding the FP32
// kernel to 64 VGPRs, so that two 1024-thread blocks share a CU, measured slower
// (35 us against 31 us on 131k Cu): the gathers then contend for the L1.
#define MD_EAM_FORCE_ARGS(R)                                                                     \
  md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,                  \
      const int* __restrict__ nneigh, int npad, const R* __restrict__ ftab_g, TabGeom g, R rc2, \
      R *force, double *vel, double inv_mass, double half_dt, DriftArgs dr,                     \
      const double *partial, const uint4 *rec, long long *ev, int ev_cap, md_ctl_dev *ctl
// THERMO: the fused kick-drift starts with the Langevin update (a kernel of its own, so
// that the random numbers do not raise the register budget of the NVE kernels).
template <int LANES, bool EV, bool TLDS, typename E, bool THERMO>
__global__ __launch_bounds__(FBLOCK) void k_eam_force_f32(
    MD_EAM_FORCE_ARGS(float)) {
  eam_force_body<float, LANES, EV, TLDS, E, THERMO>(b, pos, neigh, nneigh, npad, ftab_g, g, rc2,
                                                    force, vel, inv_mass, half_dt, dr, partial,
                                                    rec, ev, ev_cap, ctl);
}
template <int LANES, bool EV, bool TLDS, typename E, bool THERMO>
__global__ __launch_bounds__(FBLOCK) void k_eam_force_f64(MD_EAM_FORCE_ARGS(double)) {
  eam_force_body<double, LANES, EV, TLDS, E, THERMO>(b, pos, neigh, nneigh, npad, ftab_g, g, rc2,
                                                     force, vel, inv_mass, half_dt, dr, partial,
                                                     nullptr, ev, ev_cap, ctl);
}
#undef MD_EAM_FORCE_ARGS

// Ahead of the LJ pass (one block): verify the list and advance the step counter
// (md_step_bookkeeping), and zero the record slot its blocks add into.  Doing this in
// a kernel of its own keeps the step counter and the displacement maxima fixed while
// the LJ pass runs (its fused kick-drift publishes new maxima).
__global__ __launch_bounds__(1024) void k_lj_prologue(md_batch b, long long* ev, int ev_cap,
                                                     int rec_verify, md_ctl_dev* ctl) {
  md_step_bookkeeping(ctl, rec_verify != 0);
  if (ev) zero_record(b, ev, ev_cap, ctl->step_next);
}

// ---------------------------------------------------------------------------
// Lennard-Jones: U = 4 eps [(s/r)^12 - (s/r)^6] - U(r_c), one pass.
// ---------------------------------------------------------------------------
struct LJc {
  double sig2, eps4, eps24, ucut;
};

template <typename R, int LANES, bool EV, typename E, bool THERMO>
__global__ __launch_bounds__(FBLOCK) void k_lj(
    md_batch b, const double4* __restrict__ pos, const int* __restrict__ neigh,
    const int* __restrict__ nneigh, int npad, LJc c, R rc2, R* force, double* vel,
    double inv_mass, double half_dt, DriftArgs dr, const uint4* __restrict__ rec, long long* ev,
    int ev_cap, md_ctl_dev* ctl) {
  constexpr int U = 4;
  __shared__ double sh[MD_EV_LEN * 16];
  __shared__ double tsum[MD_EV_LEN * 16];
  const Slot S = force_slot<LANES>(b.n_tiles);
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // E, W xx yy zz xy xz yz, K
  const R sig2 = (R)c.sig2, eps4 = (R)c.eps4, eps24 = (R)c.eps24, ucut = (R)c.ucut;
  R fx = 0, fy = 0, fz = 0, e = 0;
  R w[6] = {0, 0, 0, 0, 0, 0};
  int i = -1, nn = 0, raw = 0;
  md_tile T{0, 0, 0, 0};
  if (S.t >= 0) {
    T = b.tiles[S.t];
    if (S.a < T.count) {
      i = T.first + S.a;
      raw = nneigh[i];
      nn = raw & MD_NN_MASK;
    }
  }
  const bool wimg = __any(raw & MD_NN_IMG);
  // the pair force, energy and virial from the separation (x, y, z) = r_j - r_i
  auto lj_pair = [&](R x, R y, R z) {
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
  if (i >= 0) {
    const E e0 = (E)i * LANES + S.l, stride = (E)npad * LANES;
    if constexpr (std::is_same<R, float>::value) {
      // FP32: separations from the 16-byte fixed-point records (minimum image by 32-bit
      // wrap-around, one load per neighbour), as in the EAM passes
      const FixBox X = fix_box(b.domains[T.rep], b.r_ns);
      const uint4 ri = rec[i];
      visit_list<LANES, U>(neigh, e0, stride, S.l, nn, [&](int j) { return load_rec16(rec, j); },
                           [&](uint4 q) {
                             float x, y, z;
                             fix_sep<false>(q, ri, X, x, y, z);
                             lj_pair(x, y, z);
                           });
    } else {
      const Img D(&b.domains[T.rep]);
      const double4 pi = pos[i];
      auto run = [&](auto img_tag) {
        constexpr bool IMG = decltype(img_tag)::value;
        visit_list<LANES, U>(neigh, e0, stride, S.l, nn,
                             [&](int j) { return load_rec(pos, j); }, [&](double4 pj) {
                               Sep sh;
                               const Sep d = separation<IMG>(D, pj, pi, sh);
                               lj_pair(d.x, d.y, d.z);
                             });
      };
      if (wimg) run(std::true_type{});
      else run(std::false_type{});
    }
  }
  fx = md_group_sum<LANES>(fx);
  fy = md_group_sum<LANES>(fy);
  fz = md_group_sum<LANES>(fz);
  double d2max = 0.0;
  int bad = 0;
  if (i >= 0 && S.l == 0) {
    if (dr.pos_out)
      acc[7] = fused_kick_drift<R, THERMO>(i, b.n_atoms, fx, fy, fz, force, vel, inv_mass,
                                           half_dt, pos,
                                   dr, ctl->step, b.domains[T.rep], b.r_ns, d2max, bad);
    else
      acc[7] = write_force_kick<R>(i, b.n_atoms, fx, fy, fz, force, vel, inv_mass, half_dt);
  }
  if (EV) {
    acc[0] = 0.5 * (double)e;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[1 + k] = 0.5 * (double)w[k];
    double res;
    int gg, kk;
    const int TPB = tiles_per_block<LANES>();
    const int nlb = (b.n_tiles + TPB - 1) / TPB;
    const int lb = md_remap_block(nlb);
    if (md_group_waves_sum<8>(acc, LANES, sh, res, gg, kk)) tsum[gg * MD_EV_LEN + kk] = res;
    __syncthreads();
    accumulate_record(b, TPB, lb, nlb, tsum,
                           ev + (size_t)(ctl->step % ev_cap) * b.n_rep * MD_EV_LEN);
  }
  // positions move without new records: carried records are void from here on
  if (dr.pos_out && !dr.rec_out && blockIdx.x == 0 && threadIdx.x == 0) ctl->rec_stale = 1;
  if (dr.pos_out) md_publish_dmax(d2max, bad, dr.thr2, ctl);
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------
bool nlist_ok(const md_nlist* nl) {
  if (!nl || !nl->neigh || !nl->nneigh) return false;
  const int L = nl->lanes;
  if (L != 1 && L != 2 && L != 4 && L != 8 && L != 16) return false;
  const int B = block_threads(*nl);
  if ((B != 256 && B != 512 && B != 1024) || B < 64 * L) return false;
  return nl->max_neigh >= L && nl->max_neigh % L == 0;
}

// Lists of 2^30 entries or more (4 GiB) take 64-bit entry offsets in the passes.
bool md_big_list(const md_nlist& nl, int npad) {
  return (size_t)nl.max_neigh * (size_t)npad >= ((size_t)1 << 30);
}

// Pair tables are staged in LDS when they fit beside the kernels' static LDS: the
// FP32 rows of the r^2 grid (62.5 KB) and the FP64 rows of 2000-point splines
// (125 KB; gfx950 has 160 KB of LDS per CU).  Read through the caches instead, the
// FP64 rows cost four vector-memory lookups per pair, which bound the FP64 passes by
// the L1 tag rate.
constexpr size_t MD_LDS_TABLE_MAX = 144 * 1024;
template <typename R>
bool table_in_lds(int nrows, int width) {
  return (size_t)nrows * width * sizeof(R) <= MD_LDS_TABLE_MAX;
}

// Dynamic LDS above 64 KB is allowed per kernel function, once.
int allow_big_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return MD_OK;
  static std::mutex mu;
  static std::vector<const void*> done;
  std::lock_guard<std::mutex> lock(mu);
  for (const void* f : done)
    if (f == fn) return MD_OK;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)MD_LDS_TABLE_MAX) !=
      hipSuccess)
    return MD_ERR_HIP;
  done.push_back(fn);
  return MD_OK;
}

template <typename R, int LANES>
int launch_eam(const md_batch& b, const md_eam& p, const char* tab, const md_table_layout& TL,
                const double* pos, const md_nlist& nl, const double* jac, void* force,
                double* saved, double* vel, double inv_mass, double half_dt, const DriftArgs& dr,
                long long* ev, int ev_cap, double* partial, uint4* rec_ws, md_ctl_dev* ctl,
                hipStream_t st) {
  // FP32: fixed-point records, carried over (md_drift.rec_in) or in the workspace
  uint4* rec = std::is_same<R, float>::value ? (dr.rec_in ? dr.rec_in : rec_ws) : nullptr;
  TabGeom g;
  g.r_lo = p.rho.x_lo;
  g.r_inv_h = 1.0 / p.rho.h;
  g.e_lo = p.emb.x_lo;
  g.e_inv_h = 1.0 / p.emb.h;
  g.nr = p.rho.ncoef - 3;
  g.ne = p.emb.ncoef - 3;
  const md_qgrid qg = md_qgrid_plan(&p);
  g.q_lo = qg.q_lo;
  g.q_inv_h = 1.0 / qg.h;
  const R rc2 = (R)(p.r_cut * p.r_cut);
  const int bt = block_threads(nl), TPB = bt / (64 * LANES);
  const dim3 grid(md_grid_blocks((b.n_tiles + TPB - 1) / TPB)), block(bt);
  const int npad = md_npad(b.n_atoms);
  const R* rtab = (const R*)(tab + TL.rtab);
  const R* ftab = (const R*)(tab + TL.ftab);
  const R* etab = (const R*)(tab + TL.etab);
  const int rows = pair_rows<R>(g);
  const bool ld = table_in_lds<R>(rows, MD_RTAB_W);
  const size_t lds_d = ld ? (size_t)rows * MD_RTAB_W * sizeof(R) : 0;
  const size_t lds_f = ld ? (size_t)rows * MD_FTAB_W * sizeof(R) : 0;
#define MD_EAM_LAUNCH(EVB, TL_, E_, TH_)                                                          \
  do {                                                                                         \
    if (jac) {                                                                                 \
      const dim3 gj((b.n_atoms + MD_ATOM_BLOCK - 1) / MD_ATOM_BLOCK), bj(MD_ATOM_BLOCK);        \
      if (p.rho.ncoef <= 64)                                                                   \
        MD_LAUNCH_TIMED(MD_KERNEL_EAM_DENSITY, (k_eam_density_jac<R, 4>), gj, bj, 0, st,        \
                        b.n_atoms, (double4*)pos, jac, p.rho.coef, p.rho.ncoef, etab, g, saved, \
                        rec, ctl);                                                             \
      else                                                                                     \
        MD_LAUNCH_TIMED(MD_KERNEL_EAM_DENSITY, (k_eam_density_jac<R, 8>), gj, bj, 0, st,        \
                        b.n_atoms, (double4*)pos, jac, p.rho.coef, p.rho.ncoef, etab, g, saved, \
                        rec, ctl);                                                             \
    } else if constexpr (std::is_same<R, float>::value) {                                      \
      if ((st_ = allow_big_lds((const void*)k_eam_density_f32<LANES, EVB, TL_, E_>, lds_d)))     \
        return st_;                                                                            \
      MD_LAUNCH_TIMED(MD_KERNEL_EAM_DENSITY, (k_eam_density_f32<LANES, EVB, TL_, E_>), grid, block, \
                      lds_d, st, b, (double4*)pos, nl.neigh, nl.nneigh, npad, rtab, etab, g,   \
                      rc2, saved, partial, rec, ev, ev_cap, dr.rec_current, ctl);              \
    } else {                                                                                   \
      if ((st_ = allow_big_lds((const void*)k_eam_density_f64<LANES, EVB, TL_, E_>, lds_d)))     \
        return st_;                                                                            \
      MD_LAUNCH_TIMED(MD_KERNEL_EAM_DENSITY, (k_eam_density_f64<LANES, EVB, TL_, E_>), grid, block, \
                      lds_d, st, b, (double4*)pos, nl.neigh, nl.nneigh, npad, rtab, etab, g,   \
                      rc2, saved, partial, rec, ev, ev_cap, 0, ctl);                           \
    }                                                                                          \
    if constexpr (std::is_same<R, float>::value) {                                             \
      if ((st_ = allow_big_lds((const void*)k_eam_force_f32<LANES, EVB, TL_, E_, TH_>, lds_f)))  \
        return st_;                                                                            \
      MD_LAUNCH_TIMED(MD_KERNEL_EAM_FORCE, (k_eam_force_f32<LANES, EVB, TL_, E_, TH_>), grid,   \
                      block,                                                                   \
                      lds_f, st, b, (const double4*)pos, nl.neigh, nl.nneigh, npad, ftab, g,   \
                      rc2, (R*)force, vel, inv_mass, half_dt, dr, partial, rec, ev, ev_cap,    \
                      ctl);                                                                    \
    } else {                                                                                   \
      if ((st_ = allow_big_lds((const void*)k_eam_force_f64<LANES, EVB, TL_, E_, TH_>, lds_f)))  \
        return st_;                                                                            \
      MD_LAUNCH_TIMED(MD_KERNEL_EAM_FORCE, (k_eam_force_f64<LANES, EVB, TL_, E_, TH_>), grid,   \
                      block,                                                                   \
                      lds_f, st, b, (const double4*)pos, nl.neigh, nl.nneigh, npad, ftab, g,   \
                      rc2, (R*)force, vel, inv_mass, half_dt, dr, partial, rec, ev, ev_cap,    \
                      ctl);                                                                    \
    }                                                                                          \
  } while (0)
  const bool big = md_big_list(nl, npad);
  int st_ = MD_OK;
  if (rec && !dr.rec_current)
    hipLaunchKernelGGL(k_fix_records, dim3(md_atom_grid(b.n_tiles)), dim3(MD_ATOM_BLOCK), 0, st, b,
                       (const double4*)pos, rec, dr.rec_in ? ctl : nullptr);
#define MD_EAM_LAUNCH_E(EVB, TL_)                                             \
  do {                                                                        \
    if (dr.L.n > 0) {                                                         \
      if (big) MD_EAM_LAUNCH(EVB, TL_, uint64_t, true);                       \
      else MD_EAM_LAUNCH(EVB, TL_, uint32_t, true);                           \
    } else {                                                                  \
      if (big) MD_EAM_LAUNCH(EVB, TL_, uint64_t, false);                      \
      else MD_EAM_LAUNCH(EVB, TL_, uint32_t, false);                          \
    }                                                                         \
  } while (0)
  if (ev) {
    if (ld) MD_EAM_LAUNCH_E(true, true);
    else MD_EAM_LAUNCH_E(true, false);
  } else {
    if (ld) MD_EAM_LAUNCH_E(false, true);
    else MD_EAM_LAUNCH_E(false, false);
  }
#undef MD_EAM_LAUNCH_E
#undef MD_EAM_LAUNCH
  return MD_OK;
}

template <typename R, int LANES>
void launch_lj(const md_batch& b, const md_lj& p, const double* pos, const md_nlist& nl,
               void* force, double* vel, double inv_mass, double half_dt, const DriftArgs& dr,
               long long* ev, int ev_cap, uint4* rec_ws, md_ctl_dev* ctl, hipStream_t st) {
  // FP32: fixed-point records, carried over (md_drift.rec_in) or in the workspace
  uint4* rec = std::is_same<R, float>::value ? (dr.rec_in ? dr.rec_in : rec_ws) : nullptr;
  LJc c;
  c.sig2 = p.sigma * p.sigma;
  c.eps4 = 4.0 * p.eps;
  c.eps24 = 24.0 * p.eps;
  const double src6 = pow(p.sigma / p.r_cut, 6.0);
  c.ucut = 4.0 * p.eps * (src6 * src6 - src6);
  const R rc2 = (R)(p.r_cut * p.r_cut);
  const int bt = block_threads(nl), TPB = bt / (64 * LANES);
  const dim3 grid(md_grid_blocks((b.n_tiles + TPB - 1) / TPB)), block(bt);
  const int npad = md_npad(b.n_atoms);
  const bool big = md_big_list(nl, npad);
#define MD_LJ_LAUNCH2(EVB, E_, TH_)                                                            \
  MD_LAUNCH_TIMED(MD_KERNEL_LJ, (k_lj<R, LANES, EVB, E_, TH_>), grid, block, 0, st, b,        \
                  (const double4*)pos, nl.neigh, nl.nneigh, npad, c, rc2, (R*)force, vel,      \
                  inv_mass, half_dt, dr, rec, ev, ev_cap, ctl)
#define MD_LJ_LAUNCH(EVB, E_)                                                                  \
  do {                                                                                         \
    if (dr.L.n > 0) MD_LJ_LAUNCH2(EVB, E_, true);                                              \
    else MD_LJ_LAUNCH2(EVB, E_, false);                                                        \
  } while (0)
  if (rec && !dr.rec_current)
    hipLaunchKernelGGL(k_fix_records, dim3(md_atom_grid(b.n_tiles)), dim3(MD_ATOM_BLOCK), 0, st, b,
                       (const double4*)pos, rec, dr.rec_in ? ctl : nullptr);
  hipLaunchKernelGGL(k_lj_prologue, dim3(1), dim3(1024), 0, st, b, ev, ev_cap,
                     rec ? dr.rec_current : 0, ctl);
  if (ev) {
    if (big) MD_LJ_LAUNCH(true, uint64_t);
    else MD_LJ_LAUNCH(true, uint32_t);
  } else {
    if (big) MD_LJ_LAUNCH(false, uint64_t);
    else MD_LJ_LAUNCH(false, uint32_t);
  }
#undef MD_LJ_LAUNCH
#undef MD_LJ_LAUNCH2
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

// The fused kick-drift's arguments (shared by the EAM and LJ passes); the force pass
// grid must fit the control block's displacement slots.
static int drift_load(const md_batch* b, const md_nlist* nl, const double* pos, double* vel,
                      double inv_mass, double half_dt, const md_drift* drift, DriftArgs* dr) {
  *dr = DriftArgs{nullptr, nullptr, 0.0, -1.0, md_walls_dev{0, 2, 0.0, 0.0, 0.0}, nullptr, nullptr,
                  0};
  if (!drift) return MD_OK;
  if (drift->rec_in && drift->rec_in == drift->rec_out) return MD_ERR_ARG;
  if (!vel || !(half_dt > 0.0) || !drift->pos_out || !drift->pos_ref ||
      drift->pos_out == pos || !isfinite(drift->dt) || half_dt != 0.5 * drift->dt)
    return MD_ERR_ARG;
  if (md_walls_load(&drift->walls, &dr->w) != MD_OK) return MD_ERR_ARG;
  if (md_langevin_load(drift->langevin, drift->dt, inv_mass, &dr->L) != MD_OK) return MD_ERR_ARG;
  dr->pos_out = (double4*)drift->pos_out;
  dr->pos_ref = drift->pos_ref;
  dr->dt = drift->dt;
  dr->thr2 = drift->half_skin < 0.0 ? -1.0 : drift->half_skin * drift->half_skin;
  dr->rec_in = (uint4*)drift->rec_in;
  dr->rec_out = (uint4*)drift->rec_out;
  dr->rec_current = drift->rec_in && drift->rec_current ? 1 : 0;
  const int tpb = block_threads(*nl) / (64 * nl->lanes);
  if (md_grid_blocks((b->n_tiles + tpb - 1) / tpb) > MD_DMAX_SLOTS) return MD_ERR_ARG;
  return MD_OK;
}

// md_eam_forces with its scratch given as pointers: the tiles' energy partials
// (8 MD_EV_LEN doubles per tile) and, in FP32, the fixed-point neighbour records (16 bytes
// per atom).  ws_ok: the caller has a workspace or scratch to pass.
static int eam_forces(const md_batch* b, const md_eam* p, md_precision prec, const void* table,
                      const double* pos, const md_nlist* nl, void* force, double* saved,
                      double* vel, double inv_mass, double half_dt, const md_drift* drift,
                      long long* ev, int ev_cap, double* partial, uint4* rec, bool ws_ok,
                      void* ctl, void* stream, const double* jac = nullptr) {
  if (!md_batch_ok(b) || !md_eam_ok(p) || !table || !pos || !nlist_ok(nl) || !force || !ws_ok ||
      !ctl)
    return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  if (ev && ev_cap < 1) return MD_ERR_ARG;
  if (vel && !(inv_mass > 0.0)) return MD_ERR_ARG;
  // FP32 takes 1-8 lanes per atom (16 is not supported)
  if (prec == MD_FP32 && nl->lanes > 8) return MD_ERR_ARG;
  DriftArgs dr;
  if (drift_load(b, nl, pos, vel, inv_mass, half_dt, drift, &dr) != MD_OK) return MD_ERR_ARG;
  if (b->n_atoms == 0 || b->n_tiles == 0) return MD_OK;
  const md_table_layout TL = md_table_plan(p, prec);
  hipStream_t st = (hipStream_t)stream;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  int rc = MD_OK;
  if (prec == MD_FP32) {
    MD_DISPATCH_LANES(nl->lanes, (rc = launch_eam<float, L_>(*b, *p, (const char*)table, TL, pos,
                                                             *nl, jac, force, saved, vel, inv_mass,
                                                             half_dt, dr, (long long*)ev, ev_cap,
                                                             partial, rec, c, st)));
  } else {
    MD_DISPATCH_LANES(nl->lanes, (rc = launch_eam<double, L_>(*b, *p, (const char*)table, TL, pos,
                                                              *nl, jac, force, saved, vel, inv_mass,
                                                              half_dt, dr, (long long*)ev, ev_cap,
                                                              partial, rec, c, st)));
  }
  if (rc != MD_OK) return rc;
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" int md_eam_forces(const md_batch* b, const md_eam* p, md_precision prec,
                             const void* table, const double* pos, const md_nlist* nl,
                             void* force, double* saved, double* vel, double inv_mass,
                             double half_dt, const md_drift* drift, long long* ev, int ev_cap,
                             void* ws, void* ctl, void* stream) {
  double* partial = nullptr;
  uint4* rec = nullptr;
  if (ws && b && b->n_atoms >= 0 && b->n_tiles >= 0) {
    const md_ws_layout WL = md_ws_plan(b);
    partial = (double*)((char*)ws + WL.partial);
    rec = (uint4*)((char*)ws + WL.rec);
  }
  return eam_forces(b, p, prec, table, pos, nl, force, saved, vel, inv_mass, half_dt, drift, ev,
                    ev_cap, partial, rec, ws != nullptr, ctl, stream);
}

extern "C" int md_eam_forces_jac(const md_batch* b, const md_eam* p, md_precision prec,
                                 const void* table, const double* pos, const md_nlist* nl,
                                 const double* jac, void* force, double* saved, void* ws,
                                 void* ctl, void* stream) {
  if (!jac || !p || p->rho.ncoef > 128) return MD_ERR_ARG;
  double* partial = nullptr;
  uint4* rec = nullptr;
  if (ws && b && b->n_atoms >= 0 && b->n_tiles >= 0) {
    const md_ws_layout WL = md_ws_plan(b);
    partial = (double*)((char*)ws + WL.partial);
    rec = (uint4*)((char*)ws + WL.rec);
  }
  return eam_forces(b, p, prec, table, pos, nl, force, saved, nullptr, 0.0, 0.0, nullptr, nullptr,
                    0, partial, rec, ws != nullptr, ctl, stream, jac);
}

// ---------------------------------------------------------------------------
// md_eam_forces_noalloc: the same passes with their scratch in a static device array.
// Layout: tile energy partials (MD_NOALLOC_MAX_TILES tiles), then the FP32 records
// (MD_NOALLOC_MAX_ATOMS atoms).  Every call on a device uses that device's one copy;
// nothing in it needs to start at zero (each pass writes what the next reads).
// ---------------------------------------------------------------------------
#define MD_NOALLOC_PARTIAL_BYTES ((size_t)MD_NOALLOC_MAX_TILES * MD_EV_LEN * sizeof(double))
#define MD_NOALLOC_REC_BYTES ((size_t)MD_NOALLOC_MAX_ATOMS * sizeof(uint4))
static __device__ __align__(256) unsigned char scratch[MD_NOALLOC_PARTIAL_BYTES +
                                                       MD_NOALLOC_REC_BYTES];

#define MD_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void* g_scratch_dev[MD_MAX_DEVICES];  // device address of `scratch` on each device

// The current device's address of `scratch`, looked up once per device (with that device
// current).  The array's name in host code is a host-side stand-in, never a device address.
static int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MD_MAX_DEVICES) return MD_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MD_ERR_HIP;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return MD_OK;
}

extern "C" int md_eam_forces_noalloc(const md_batch* b, const md_eam* p, md_precision prec,
                                     const void* table, const double* pos, const md_nlist* nl,
                                     void* force, double* saved, double* vel, double inv_mass,
                                     double half_dt, const md_drift* drift, long long* ev,
                                     int ev_cap, void* ctl, void* stream) {
  if (!md_batch_ok(b)) return MD_ERR_ARG;
  if (b->n_atoms > MD_NOALLOC_MAX_ATOMS || b->n_tiles > MD_NOALLOC_MAX_TILES)
    return MD_ERR_WORKSPACE;
  void* base = nullptr;
  const int st = scratch_address(&base);
  if (st != MD_OK) return st;
  double* partial = (double*)base;
  uint4* rec = (uint4*)((char*)base + MD_NOALLOC_PARTIAL_BYTES);
  return eam_forces(b, p, prec, table, pos, nl, force, saved, vel, inv_mass, half_dt, drift, ev,
                    ev_cap, partial, rec, true, ctl, stream);
}

extern "C" int md_lj_forces(const md_batch* b, const md_lj* p, md_precision prec,
                            const double* pos, const md_nlist* nl, void* force, double* vel,
                            double inv_mass, double half_dt, const md_drift* drift, long long* ev,
                            int ev_cap, void* ws, void* ctl, void* stream) {
  if (!md_batch_ok(b) || !p || !pos || !nlist_ok(nl) || !force || !ws || !ctl) return MD_ERR_ARG;
  if (!(p->sigma > 0.0) || !(p->r_cut > 0.0)) return MD_ERR_ARG;
  if (prec != MD_FP64 && prec != MD_FP32) return MD_ERR_ARG;
  // FP32 takes 1-8 lanes per atom, as in md_eam_forces
  if (prec == MD_FP32 && nl->lanes > 8) return MD_ERR_ARG;
  if (ev && ev_cap < 1) return MD_ERR_ARG;
  if (vel && !(inv_mass > 0.0)) return MD_ERR_ARG;
  DriftArgs dr;
  if (drift_load(b, nl, pos, vel, inv_mass, half_dt, drift, &dr) != MD_OK) return MD_ERR_ARG;
  if (b->n_atoms == 0 || b->n_tiles == 0) return MD_OK;
  hipStream_t st = (hipStream_t)stream;
  md_ctl_dev* c = (md_ctl_dev*)ctl;
  uint4* rec = (uint4*)((char*)ws + md_ws_plan(b).rec);
  if (prec == MD_FP32) {
    MD_DISPATCH_LANES(nl->lanes, (launch_lj<float, L_>(*b, *p, pos, *nl, force, vel, inv_mass,
                                                       half_dt, dr, (long long*)ev, ev_cap, rec,
                                                       c, st)));
  } else {
    MD_DISPATCH_LANES(nl->lanes, (launch_lj<double, L_>(*b, *p, pos, *nl, force, vel, inv_mass,
                                                        half_dt, dr, (long long*)ev, ev_cap, rec,
                                                        c, st)));
  }
  MD_LAUNCH_CHECK();
  return MD_OK;
}
