/*
 * A plain C client of the md950 C ABI (include/md.h): an NVE velocity-Verlet run of a
 * Lennard-Jones system (eq. 1.6) in one periodic box, with lists rebuilt on the
 * half-skin criterion (Sec. 1.4).  It uses nothing but the C declarations and the HIP
 * runtime's memory API, so it shows that the library stands on its own without
 * Python or torch.  The caller (this program) owns every buffer.
 *
 *   lj_nve <input> <output> <steps>
 *
 * input  (binary, native endianness): int32 n; float64 box_len[3], eps, sigma, r_cut,
 *        skin, mass, dt; float64 pos[n][3]; float64 vel[n][3]   (the box starts at 0)
 * output (binary): float64 record[steps + 1][2] = {E_pot, K} per step (eV); then
 *        float64 pos[n][3], vel[n][3] at the end, in the input's atom order; then int32
 *        {status, step, n_rebuilds, max_nneigh} from md_read_flags.
 * Exit status 0 on success, 1 on a usage or I/O error, 2 on a HIP or md950 error.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "md.h"

#define HIP_OK(call)                                                     \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) {                                              \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));         \
      exit(2);                                                           \
    }                                                                    \
  } while (0)

#define MD_CALL(call)                                                           \
  do {                                                                          \
    int s_ = (call);                                                            \
    if (s_ != MD_OK) {                                                          \
      fprintf(stderr, "%s: %s\n", #call, md_status_string(s_));                 \
      exit(2);                                                                  \
    }                                                                           \
  } while (0)

static void* dev_alloc(size_t bytes) {
  void* p = NULL;
  HIP_OK(hipMalloc(&p, bytes > 0 ? bytes : 256));
  HIP_OK(hipMemset(p, 0, bytes > 0 ? bytes : 256));
  return p;
}

static void read_all(FILE* f, void* dst, size_t bytes) {
  if (fread(dst, 1, bytes, f) != bytes) {
    fprintf(stderr, "input ends early\n");
    exit(1);
  }
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s <input> <output> <steps>\n", argv[0]);
    return 1;
  }
  const int steps = atoi(argv[3]);
  FILE* in = fopen(argv[1], "rb");
  if (!in || steps < 0) {
    fprintf(stderr, "cannot read %s\n", argv[1]);
    return 1;
  }
  int n;
  double hdr[9];
  read_all(in, &n, sizeof(int));
  read_all(in, hdr, sizeof(hdr));
  if (n < 1) return 1;
  double* x = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  double* v = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  read_all(in, x, sizeof(double) * 3 * (size_t)n);
  read_all(in, v, sizeof(double) * 3 * (size_t)n);
  fclose(in);
  const double eps = hdr[3], sigma = hdr[4], r_cut = hdr[5], skin = hdr[6], mass = hdr[7],
               dt = hdr[8];

  /* plan: one periodic box, cell grid for r_ns = r_cut + skin */
  md_box box;
  memset(&box, 0, sizeof(box));
  for (int a = 0; a < 3; ++a) {
    box.len[a] = hdr[a];
    box.periodic[a] = 1;
  }
  const int atom_off[2] = {0, n};
  const double r_ns = r_cut + skin;
  int n_cells, n_tiles;
  MD_CALL(md_plan_count(1, &box, atom_off, r_ns, MD_TILE_ATOMS, &n_cells, &n_tiles));
  md_domain dom;
  md_tile* tiles = (md_tile*)malloc(sizeof(md_tile) * (size_t)n_tiles);
  MD_CALL(md_plan(1, &box, atom_off, r_ns, MD_TILE_ATOMS, &dom, tiles));
  md_batch b;
  memset(&b, 0, sizeof(b));
  b.n_rep = 1;
  b.n_atoms = n;
  b.n_cells = n_cells;
  b.n_tiles = n_tiles;
  b.tile_atoms = MD_TILE_ATOMS;
  b.r_ns = r_ns;
  void* d_dom = dev_alloc(sizeof(md_domain));
  void* d_tiles = dev_alloc(sizeof(md_tile) * (size_t)n_tiles);
  HIP_OK(hipMemcpy(d_dom, &dom, sizeof(md_domain), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_tiles, tiles, sizeof(md_tile) * (size_t)n_tiles, hipMemcpyHostToDevice));
  b.domains = (const md_domain*)d_dom;
  b.tiles = (const md_tile*)d_tiles;

  /* atom arrays: positions as double4 records, velocities and forces [3][n] */
  double* h4 = (double*)calloc(4 * (size_t)n, sizeof(double));
  double* hv = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  int* hid = (int*)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      h4[4 * i + a] = x[3 * i + a];
      hv[(size_t)a * n + i] = v[3 * i + a];
    }
    hid[i] = i;
  }
  double* pos = (double*)dev_alloc(sizeof(double) * 4 * (size_t)n);
  double* vel = (double*)dev_alloc(sizeof(double) * 3 * (size_t)n);
  double* force = (double*)dev_alloc(sizeof(double) * 3 * (size_t)n);
  double* pos_ref = (double*)dev_alloc(sizeof(double) * 3 * (size_t)n);
  int* id = (int*)dev_alloc(sizeof(int) * (size_t)n);
  int* cell_start = (int*)dev_alloc(sizeof(int) * ((size_t)n_cells + 1));
  HIP_OK(hipMemcpy(pos, h4, sizeof(double) * 4 * (size_t)n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(vel, hv, sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(id, hid, sizeof(int) * (size_t)n, hipMemcpyHostToDevice));
  void* ws = dev_alloc(md_workspace_bytes(&b));
  void* ctl = dev_alloc(md_ctl_bytes());
  const int lanes = 4, max_neigh = 128;
  const size_t npad = ((size_t)n + 63) / 64 * 64;
  md_nlist nl;
  nl.neigh = (int*)dev_alloc(sizeof(int) * (size_t)max_neigh * npad);
  nl.nneigh = (int*)dev_alloc(sizeof(int) * (size_t)n);
  nl.max_neigh = max_neigh;
  nl.lanes = lanes;
  nl.block = 0; /* the default launch shape */
  const int cap = steps + 1;
  long long* ev = (long long*)dev_alloc(sizeof(long long) * MD_EV_LEN * (size_t)cap);
  md_lj lj = {eps, sigma, r_cut};
  const double inv_mass = 1.0 / mass;
  void* stream = NULL;

  /* step 0: lists and forces at the initial positions (kinetic energy, no kick) */
  MD_CALL(md_ctl_init(ctl, stream));
  MD_CALL(md_bin_cells(&b, MD_ALWAYS, pos, vel, id, pos_ref, cell_start, ws, ctl, stream));
  MD_CALL(md_build_neighbors(&b, MD_ALWAYS, pos, cell_start, &nl, ctl, stream));
  MD_CALL(md_lj_forces(&b, &lj, MD_FP64, pos, &nl, force, vel, inv_mass, 0.0, NULL, ev, cap,
                       ws, ctl, stream));
  /* steps 1..steps: kick-drift, rebuild when an atom moved half the skin, forces + kick */
  for (int s = 1; s <= steps; ++s) {
    MD_CALL(md_verlet_step(&b, MD_KICK_DRIFT, dt, pos, vel, force, MD_FP64, inv_mass, NULL, NULL,
                           pos_ref, 0.5 * skin, ctl, stream));
    MD_CALL(md_bin_cells(&b, MD_IF_FLAGGED, pos, vel, id, pos_ref, cell_start, ws, ctl, stream));
    MD_CALL(md_build_neighbors(&b, MD_IF_FLAGGED, pos, cell_start, &nl, ctl, stream));
    MD_CALL(md_lj_forces(&b, &lj, MD_FP64, pos, &nl, force, vel, inv_mass, 0.5 * dt, NULL, ev,
                         cap, ws, ctl, stream));
  }
  int flags[4];
  const int status = md_read_flags(ctl, flags, stream);
  HIP_OK(hipDeviceSynchronize());

  /* results, back in the input's atom order */
  long long* hev = (long long*)malloc(sizeof(long long) * MD_EV_LEN * (size_t)cap);
  HIP_OK(hipMemcpy(hev, ev, sizeof(long long) * MD_EV_LEN * (size_t)cap, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(h4, pos, sizeof(double) * 4 * (size_t)n, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(hv, vel, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(hid, id, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    const int o = hid[i];
    if (o < 0 || o >= n) return 2;
    for (int a = 0; a < 3; ++a) {
      x[3 * o + a] = h4[4 * i + a];
      v[3 * o + a] = hv[(size_t)a * n + i];
    }
  }
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 1;
  for (int s = 0; s <= steps; ++s) {
    const double e[2] = {(double)hev[(size_t)s * MD_EV_LEN] / MD_EV_SCALE,
                         (double)hev[(size_t)s * MD_EV_LEN + 7] / MD_EV_SCALE};
    fwrite(e, sizeof(double), 2, out);
  }
  fwrite(x, sizeof(double), 3 * (size_t)n, out);
  fwrite(v, sizeof(double), 3 * (size_t)n, out);
  const int tail[4] = {status, flags[1], flags[2], flags[3]};
  fwrite(tail, sizeof(int), 4, out);
  fclose(out);
  printf("lj_nve: %d atoms, %d steps, %d rebuilds, status %s\n", n, steps, flags[2],
         md_status_string(status));
  return status == MD_OK ? 0 : 2;
}
