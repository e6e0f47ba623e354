/*
 * md.h - C ABI of the MI355X (gfx950) short-range molecular-dynamics hot path.
 *
 * The library integrates Newton's equations m_i r_i'' = f_i = -grad_i U
 * (MDcraft paper, Sec. 1.5, eq. 1.5) with velocity Verlet for atoms that
 * interact through short-range potentials (Sec. 1.6: Lennard-Jones and
 * single-element EAM), using a cell grid and Verlet neighbour lists with a
 * skin (Sec. 1.4, eq. 1.2) in periodic or walled boxes (Sec. 1.5).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *     owns all memory; the library never allocates.  Sizes come from the
 *     md_*_bytes() queries.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *     default stream) and is stream-ordered.  No entry point synchronises
 *     except md_read_flags().  Calls on distinct streams with distinct buffers
 *     are independent; calls that share a control block must be ordered.
 *   - Units: angstrom, eV, ps, u (atomic mass), K.  Accelerations use
 *     1 eV/(u angstrom) = 9648.5332157 angstrom/ps^2.
 *   - Atom arrays hold n_atoms entries of all boxes of a batch end to end.
 *     Positions are `double4` records {x, y, z, w} ([n_atoms][4] doubles); the
 *     w slot is library scratch (the EAM passes store F'(rhobar) there).
 *     Velocities and forces are structure-of-arrays [3][n_atoms] (x block, y
 *     block, z block).  Positions and velocities are always FP64; forces are
 *     FP64 or FP32 as the precision argument says.
 *   - After md_bin_cells the atoms are in cell order inside each box; id[]
 *     carries the caller's original atom ids along with the permutation.
 *     Positions are wrapped into the box at that point only; between rebuilds
 *     an atom may stand outside its periodic box by at most half the skin.
 *   - A batch may hold no atoms (n_atoms = 0, n_tiles = 0, tiles may then be
 *     NULL; a box of a batch may be empty too).  With n_atoms = 0 every entry
 *     point checks its arguments and returns MD_OK without enqueuing work, except
 *     md_profiles, md_eam_backward, md_eam_backward_jac and md_force_loss, which still
 *     write their (zero) results.
 *   - Return values are md_status codes.  Argument errors return at once and
 *     enqueue nothing.  Conditions detected on the device set sticky bits in
 *     the control block; md_read_flags() reads and maps them.
 */
#ifndef MD950_MD_H
#define MD950_MD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MD_OK = 0,
  MD_ERR_ARG = -1,            /* bad argument (null pointer, size, enum) */
  MD_ERR_BOX = -2,            /* r_ns >= L/2 on a periodic axis, or an empty box */
  MD_ERR_NEIGH_OVERFLOW = -3, /* an atom has more than max_neigh neighbours */
  MD_ERR_TABLE_RANGE = -4,    /* r below a table's start or rhobar outside the F table */
  MD_ERR_WALL = -5,           /* an atom left a non-periodic extent */
  MD_ERR_NONFINITE = -6,      /* a position became NaN or infinite */
  MD_ERR_HIP = -7,            /* a HIP runtime call failed */
  MD_ERR_WORKSPACE = -8,      /* workspace or capacity too small */
  MD_ERR_STALE_LIST = -9,     /* an atom moved more than half the skin since the last list
                                 build and no rebuild followed (forces may miss pairs) */
  MD_ERR_STALE_RECORDS = -10  /* a force call was told its carried FP32 neighbour records
                                 were current (md_drift.rec_current) after positions had
                                 changed otherwise */
} md_status;

/* Device flag bits (md_read_flags output). */
#define MD_FLAG_NEIGH_OVERFLOW 1
#define MD_FLAG_TABLE_RANGE 2
#define MD_FLAG_WALL 4
#define MD_FLAG_NONFINITE 8
#define MD_FLAG_STALE_LIST 16
#define MD_FLAG_STALE_RECORDS 32

typedef enum { MD_FP64 = 0, MD_FP32 = 1 } md_precision; /* MD_FP32: FP32 pair math and
                                                          force accumulation, FP64
                                                          positions/integration/reductions */

typedef enum { MD_ALWAYS = 0, MD_IF_FLAGGED = 1 } md_rebuild_mode;
typedef enum { MD_KICK_DRIFT = 0, MD_KICK = 1 } md_verlet_phase;

/* Orthorhombic box [lo, lo + len) per axis (host struct). */
typedef struct md_box {
  double lo[3];
  double len[3];
  int periodic[3];
  int pad;
} md_box;

/* Per-box cell grid and bookkeeping, produced by md_plan (device array of n_rep). */
typedef struct md_domain {
  double lo[3];
  double len[3];
  double inv_len[3];
  double inv_w[3]; /* cells per unit length, nc / len */
  int nc[3];
  int periodic[3];
  int cell_off; /* first global cell index of this box */
  int atom_off; /* first atom */
  int n_atoms;
  int tile_off; /* first work tile */
  int n_tiles;
  int pad;
} md_domain;

/* A work tile: up to tile_atoms consecutive atoms of one box.  The kernels take
 * tiles of MD_TILE_ATOMS atoms (one wavefront at one lane per atom). */
#define MD_TILE_ATOMS 64
typedef struct md_tile {
  int rep;
  int first;
  int count;
  int pad;
} md_tile;

/* A batch of independent boxes laid end to end.  A single system is n_rep = 1. */
typedef struct md_batch {
  int n_rep;
  int n_atoms;
  int n_cells;
  int n_tiles;
  int tile_atoms;
  int pad;
  double r_ns;              /* neighbour search radius the grids were planned for */
  const md_domain* domains; /* device [n_rep] */
  const md_tile* tiles;     /* device [n_tiles] */
} md_batch;

/* Neighbour-list layout: padded ELL, strided for `lanes` lanes per atom.  Entry
 * n of atom i lives at index ((n / lanes) * n_atoms_pad + i) * lanes + n % lanes
 * of an int32 array of max_neigh * n_atoms_pad entries, n_atoms_pad = n_atoms
 * rounded up to 64.  Entries are atom indices in the current (cell) order. */
typedef struct md_nlist {
  int* neigh;   /* device [max_neigh * n_atoms_pad] */
  int* nneigh;  /* device [n_atoms]: list length in bits 0..29; bit 30 (MD_NN_IMG) set when
                   the atom's 3x3x3 cell block crosses a periodic boundary */
  int max_neigh;/* multiple of lanes */
  int lanes;    /* 1, 2, 4, 8 or 16 */
  int block;    /* threads per workgroup of the force passes (the atoms one workgroup takes,
                   block / lanes, are its task): 0 (= 1024), 256, 512 or 1024, at least
                   64 * lanes; MD_ERR_ARG otherwise.  A launch-shape choice only: results
                   do not depend on it beyond the rounding order of the per-box records. */
} md_nlist;

#define MD_NN_IMG (1 << 30)

/* Uniform cubic B-spline on breakpoints x_lo + k h (k = 0..ncoef-3): ncoef
 * coefficients (FP64, device). */
typedef struct md_spline {
  const double* coef;
  int ncoef;
  int pad;
  double x_lo;
  double h;
} md_spline;

/* Single-element EAM: pair phi(r), density rho(r), embedding F(rhobar); phi and rho
 * must share one grid.  Interaction for r < r_cut only. */
typedef struct md_eam {
  md_spline phi, rho, emb;
  double r_cut;
} md_eam;

typedef struct md_lj {
  double eps;
  double sigma;
  double r_cut; /* energy shifted by U(r_cut); force unshifted */
} md_lj;

/* A piston plane at z0 + v t along `axis`, reflecting specularly in its frame,
 * and a static top wall at top (Sec. 1.5, hard walls). */
typedef struct md_walls {
  int enabled;
  int axis;
  double piston_z0;
  double piston_v;
  double top;
} md_walls;

/* Langevin thermostat (Sec. 1.5: a Langevin force added to eq. 1.5 gives the NVT
 * ensemble; Sec. 3.1 thermostats slabs of the sample, each with a target
 * temperature, a mean velocity and a stiffness).  In each region the equation of
 * motion gains -m gamma (v - u) + sqrt(2 m gamma k_B T) eta(t).  Discretisation:
 * the exact Ornstein-Uhlenbeck velocity update over dt, applied at the start of
 * md_verlet_step(MD_KICK_DRIFT) before the half kick (the OBABO splitting of
 * Bussi and Parrinello, Phys. Rev. E 75, 056707 (2007), with its two half-step
 * O parts merged):
 *   v <- u + c1 (v - u) + c2 xi,  c1 = exp(-gamma dt),  c2 = sqrt((1 - c1^2) k_B T / m).
 * xi holds three standard normals per atom and step from Philox4x32-10 (Salmon,
 * Moraes, Dror and Shaw, SC'11) with counter {id, step, 0, 0} and key {seed low
 * 32 bits, seed high 32 bits}, by the Box-Muller transform of its four words
 * w0..w3: with U_k = (w_k + 1) 2^-32 for k = 0, 2 and U_k = w_k 2^-32 for
 * k = 1, 3, xi_x = sqrt(-2 ln U_0) cos(2 pi U_1), xi_y = sqrt(-2 ln U_0)
 * sin(2 pi U_1), xi_z = sqrt(-2 ln U_2) cos(2 pi U_3).  step is the number of the
 * step being started (the control block's step + 1), id the atom's original id,
 * so the noise does not depend on the cell order.  An atom belongs to the first
 * region with lo <= x[axis] < hi, x at the start of the step and, on a periodic
 * axis, folded into the box as md_bin_cells wraps it; atoms outside every region
 * follow plain velocity Verlet. */
#define MD_MAX_THERMO_REGIONS 4
typedef struct md_thermo_region {
  double lo, hi;       /* slab along md_langevin.axis, angstrom (+-HUGE_VAL: unbounded) */
  double temperature;  /* K, >= 0 */
  double gamma;        /* friction (stiffness), 1/ps, >= 0 */
  double u[3];         /* mean velocity, angstrom/ps */
} md_thermo_region;
typedef struct md_langevin {
  const int* id;       /* device [n]: original atom ids (md_bin_cells keeps them in step) */
  unsigned long long seed;
  int axis;            /* 0, 1 or 2 */
  int n_regions;       /* 1 .. MD_MAX_THERMO_REGIONS */
  md_thermo_region region[MD_MAX_THERMO_REGIONS];
} md_langevin;

/* Per-step thermodynamic record per box: {E_pot, W_xx, W_yy, W_zz, W_xy, W_xz,
 * W_yz, K}, W the pair virial 1/2 sum_ij r_ij f_ij (Appendix), K the kinetic
 * energy (eq. 1.3).  Stored as signed 64-bit fixed point, MD_EV_SCALE units per
 * eV (resolution 1.5e-11 eV, range +-1.3e8 eV): blocks add their sums with
 * integer atomics, so the records are reproducible bit for bit. */
#define MD_EV_LEN 8
#define MD_EV_SCALE 68719476736.0 /* 2^36 */

/* ---------------------------------------------------------------------------
 * Set-up (host)
 * ------------------------------------------------------------------------- */

/* Count the cells and tiles a batch needs.  Host arrays: boxes[n_rep],
 * atom_off[n_rep + 1] (atom_off[0] = 0, box r holds atoms atom_off[r] ..
 * atom_off[r + 1] - 1); tile_atoms must be MD_TILE_ATOMS.  Returns MD_ERR_BOX if a periodic length is not above
 * 2 r_ns (the minimum image of every neighbour must be unique), MD_ERR_ARG if
 * the batch holds more than MD_MAX_ATOMS atoms (the passes address the 32-byte
 * position records with 32-bit byte offsets). */
#define MD_MAX_ATOMS ((1 << 27) - 64)
int md_plan_count(int n_rep, const md_box* boxes, const int* atom_off, double r_ns,
                  int tile_atoms, int* n_cells, int* n_tiles);

/* Fill the host arrays domains[n_rep] and tiles[n_tiles] (sizes from
 * md_plan_count).  The cell grid of each box has nc = max(1, floor(len / r_ns))
 * cells per axis, so a cell edge is at least r_ns (Sec. 1.4: a virtual grid
 * with cell edge R).  The caller copies both arrays to the device and fills an
 * md_batch with them. */
int md_plan(int n_rep, const md_box* boxes, const int* atom_off, double r_ns, int tile_atoms,
            md_domain* domains, md_tile* tiles);

/* Bytes of the device control block (step counter, rebuild flag, error flags,
 * reduction counters).  md_ctl_init clears it (by a kernel, graph safe). */
size_t md_ctl_bytes(void);
int md_ctl_init(void* ctl, void* stream);

/* Bytes of workspace md_bin_cells and the force passes need for this batch. */
size_t md_workspace_bytes(const md_batch* b);

/* Bytes of the packed interval tables md_eam_prepare writes. */
size_t md_eam_table_bytes(const md_eam* p, md_precision prec);

/* Complete (clamped) cubic spline fit on the device: given K samples y[k] of a
 * function at x_lo + k h and its end slopes, write the K + 2 B-spline
 * coefficients that interpolate every sample and match both slopes (the form
 * in which a tabulated potential file is turned into a spline; Sec. 3.3). */
int md_spline_fit(const double* y, int K, double h, double dy_lo, double dy_hi, double* coef,
                  void* stream);

/* Convert EAM B-spline coefficients into per-interval polynomial tables in the
 * given precision (values and derivatives in Horner form).  Call again whenever
 * the coefficients change. */
int md_eam_prepare(const md_eam* p, md_precision prec, void* table, void* stream);

/* ---------------------------------------------------------------------------
 * Hot path (Sec. 1.4 - 1.6)
 * ------------------------------------------------------------------------- */

/* Wrap positions into their boxes, bin atoms into the cell grid (a counting
 * sort, Sec. 1.4 "bucket sort"), and permute pos, vel and id into cell order
 * (order inside a cell: ascending id).  Sets pos_ref = pos (the reference of
 * the displacement check).  cell_start[n_cells + 1] receives the first atom of
 * each cell.  With MD_IF_FLAGGED the kernels do nothing unless the last
 * md_verlet_step found a displacement above half the skin (rebuild on the
 * threshold, Sec. 1.4); MD_ALWAYS rebuilds unconditionally (e.g. every k steps,
 * as in the benchmark of Sec. 1.7).  Either way the first force pass after a
 * kick-drift verifies the criterion and sets MD_FLAG_STALE_LIST if an atom moved
 * more than half the skin since the list was built. */
int md_bin_cells(const md_batch* b, md_rebuild_mode mode, double* pos, double* vel, int* id,
                 double* pos_ref, int* cell_start, void* ws, void* ctl, void* stream);

/* Build the full Verlet list {j != i : |r_ij| < r_ns} (Sec. 1.4, eq. 1.2 with
 * r_ns = r_c + skin) by scanning the 3x3x3 block of cells around each atom's
 * cell (de-duplicated when a box has fewer than 3 cells on an axis).  Distances
 * use the minimum image in FP64 with no fused multiply-add, so the set equals
 * the brute-force definition bit for bit.  Each list is in candidate order
 * (stencil cell, then position in the cell), so lists are reproducible run to
 * run.  Sets MD_FLAG_NEIGH_OVERFLOW when an atom has more than max_neigh
 * neighbours (the first max_neigh are kept). */
int md_build_neighbors(const md_batch* b, md_rebuild_mode mode, const double* pos,
                       const int* cell_start, const md_nlist* nl, void* ctl, void* stream);

/* The next step's kick-drift fused into a force pass (md_lj_forces, md_eam_forces):
 * after the trailing
 * half kick of step n, v += dt/2 f/m and x_out = x + dt v with the walls at
 * t = (step + 1) dt, then the half-skin displacement check against pos_ref --
 * the same operations, in the same order, as md_verlet_step(MD_KICK_DRIFT) at
 * the start of step n + 1 (Sec. 1.5), saving its pass over the atoms.  pos_out
 * (double4 [n], device) must not be pos: other atoms still read pos in the same
 * pass; the caller swaps the two buffers after the call.  Velocities are left at
 * the half step n + 1/2; the record of step n holds the kinetic energy at v(n).
 * The force pass keeps one displacement slot per block: MD_ERR_ARG when its grid of
 * ceil(n_tiles * lanes / 16) blocks (rounded up to a multiple of 8) exceeds
 * MD_DRIFT_MAX_BLOCKS.
 *
 * FP32 neighbour records carried from step to step (MD_FP32 only; both NULL otherwise
 * ignored).  The FP32 passes gather 16-byte records per atom (32-bit fixed-point x, y, z
 * and F'), which a call normally makes from pos in its workspace.  rec_out (device,
 * 16-byte aligned, 16 n bytes): the fused kick-drift also writes the records of pos_out
 * there.  rec_in: the records of pos, as an earlier call wrote them to its rec_out; the
 * call then uses that buffer instead of its workspace's (writing F' into it) and remakes
 * the records from pos only when positions changed since by anything else the library
 * does -- md_ctl_init, md_bin_cells reordering the atoms, md_verlet_step's drift -- which
 * the control block records on the device.  The caller owns this contract: positions
 * written outside the library since that earlier call void rec_in (pass NULL, or call
 * md_ctl_init).  rec_in and rec_out must be different buffers (MD_ERR_ARG).
 * rec_current = 1 declares more: that nothing changed positions since the call that wrote
 * rec_in (no md_bin_cells, md_verlet_step or md_ctl_init in between), so the call does not
 * even launch the check; should the control block say otherwise, the records are still
 * used as they are and MD_FLAG_STALE_RECORDS is raised (md_read_flags then returns
 * MD_ERR_STALE_RECORDS and the step is void).
 *
 * langevin (NULL: NVE): the Langevin velocity update of md_verlet_step (NVT, Sec. 1.5)
 * applied to v(n) before the next half kick, with the random numbers of step n + 1 --
 * the same operations as md_verlet_step(MD_KICK_DRIFT, ..., langevin) at the start of
 * step n + 1; MD_ERR_ARG for a malformed md_langevin (as md_verlet_step). */
#define MD_DRIFT_MAX_BLOCKS 32768
typedef struct md_drift {
  double* pos_out;
  const double* pos_ref; /* [3][n] */
  double dt;
  double half_skin;      /* < 0: no criterion */
  md_walls walls;        /* walls.enabled = 0: none */
  void* rec_in;          /* FP32 neighbour records of pos, or NULL */
  void* rec_out;         /* FP32 neighbour records of pos_out are written here, or NULL */
  int rec_current;       /* 1: rec_in is known to be current (see above); 0: checked */
  int pad;
  const md_langevin* langevin; /* thermostat of the next kick, or NULL (see above) */
} md_drift;

/* Lennard-Jones forces (eq. 1.6), energy and virial.  force is [3][n] FP64 or
 * FP32.  If vel is not NULL the trailing half kick v += half_dt f / m is applied
 * and the kinetic energy is reduced.  If ev is not NULL the per-box record
 * {E, W[6], K} is written to ev[(step % ev_cap) * n_rep + rep] (step = the
 * control block's step counter).  drift: NULL, or the next step's kick-drift to
 * fuse (md_drift, as for md_eam_forces).  MD_FP32 takes lists with 1, 2, 4 or 8
 * lanes per atom (16: MD_ERR_ARG); MD_FP64 all five. */
int md_lj_forces(const md_batch* b, const md_lj* p, md_precision prec, const double* pos,
                 const md_nlist* nl, void* force, double* vel, double inv_mass, double half_dt,
                 const md_drift* drift, long long* ev, int ev_cap, void* ws, void* ctl,
                 void* stream);


/* EAM forces (Sec. 1.6: the pair force of eq. 1.6 with the embedded-atom energy,
 * Sec. 3.3: the potential given as tables): a density pass (rhobar_i = sum_j rho(r_ij), F(rhobar_i),
 * F'(rhobar_i), the energy) then a force pass
 *   f_i = -sum_j [phi'(r) + (F'(rhobar_i) + F'(rhobar_j)) rho'(r)] r_ij / r,
 * with the virial and an optional trailing half kick as in md_lj_forces.
 * table: from md_eam_prepare in the same precision.  If saved is not NULL it
 * receives {rhobar, F', F''} as [3][n] FP64 for md_eam_backward.  MD_FP32 takes
 * lists with 1, 2, 4 or 8 lanes per atom (16: MD_ERR_ARG); MD_FP64 all five.
 * drift: NULL, or the next step's kick-drift to fuse (md_drift; requires vel and
 * half_dt = dt / 2). */
int md_eam_forces(const md_batch* b, const md_eam* p, md_precision prec, const void* table,
                  const double* pos, const md_nlist* nl, void* force, double* saved,
                  double* vel, double inv_mass, double half_dt, const md_drift* drift,
                  long long* ev, int ev_cap, void* ws,
                  void* ctl, void* stream);

/* md_eam_forces without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as md_eam_forces, minus ws; the scratch
 * (tile energy partials and the FP32 neighbour records) lives in a static device array of
 * the library, MD_NOALLOC_MAX_TILES * 64 + MD_NOALLOC_MAX_ATOMS * 16 bytes (18 MiB), one
 * copy per GPU, held until the process ends.  Batches with more than MD_NOALLOC_MAX_ATOMS
 * atoms or MD_NOALLOC_MAX_TILES tiles return MD_ERR_WORKSPACE.  The call allocates nothing;
 * its first call on a device looks up that device's copy of the array (hipGetSymbolAddress).
 * All calls on one GPU share the array: calls that overlap on one GPU (on different streams
 * or from different threads without ordering) race. */
#define MD_NOALLOC_MAX_ATOMS (1 << 20)
#define MD_NOALLOC_MAX_TILES 32768
int md_eam_forces_noalloc(const md_batch* b, const md_eam* p, md_precision prec,
                          const void* table, const double* pos, const md_nlist* nl, void* force,
                          double* saved, double* vel, double inv_mass, double half_dt,
                          const md_drift* drift, long long* ev, int ev_cap, void* ctl,
                          void* stream);

/* Velocity Verlet (Sec. 1.5).  MD_KICK_DRIFT: the Langevin update if lang is not
 * NULL (md_langevin), then v += half_dt f/m; x += dt v; walls at t = (step + 1) dt;
 * per-block maxima of |x - pos_ref|^2 are kept for the rebuild decision (compared
 * with half_skin^2; half_skin < 0: no criterion).  The step counter advances in
 * the next force pass.  MD_KICK: v += half_dt f/m only (lang must be NULL).
 * MD_ERR_ARG for a malformed md_langevin (region count, axis, negative T or
 * gamma, NULL id). */
int md_verlet_step(const md_batch* b, md_verlet_phase phase, double dt, double* pos,
                   double* vel, const void* force, md_precision prec, double inv_mass,
                   const md_walls* walls, const md_langevin* lang, const double* pos_ref,
                   double half_skin, void* ctl, void* stream);

/* Density Jacobian of fixed positions for the EAM of Sec. 1.6: jac[i][k] = d rhobar_i /
 * d c_rho_k = sum_j beta_k(r_ij) over the pairs of atom i within r_cut (rhobar is linear
 * in the density coefficients, so jac depends on the positions, the list, the rho grid and
 * r_cut, not on coefficient values).  jac: [n][rho.ncoef] FP64, row-major, current atom
 * order, md_density_jacobian_bytes(b, p) bytes, overwritten.  rho.ncoef at most 128
 * (bytes 0 and MD_ERR_ARG otherwise).  Deterministic.  Table-range flag as the forces. */
size_t md_density_jacobian_bytes(const md_batch* b, const md_eam* p);
int md_eam_density_jacobian(const md_batch* b, const md_eam* p, const double* pos,
                            const md_nlist* nl, double* jac, void* ctl, void* stream);

/* md_eam_forces (no kick, drift or energy records) for fixed positions whose density
 * Jacobian `jac` (md_eam_density_jacobian: same positions, list, rho grid and r_cut) is
 * kept: the density pass becomes rhobar = jac c_rho, one row per atom, in place of a
 * visit of every list; the force pass is the same.  force, saved, ws and the table as in
 * md_eam_forces.  rhobar and so F', F'' agree with md_eam_forces to rounding (FP64; in
 * FP32 to the resampled tables' error).  MD_ERR_ARG for a NULL jac or rho.ncoef > 128. */
int md_eam_forces_jac(const md_batch* b, const md_eam* p, md_precision prec, const void* table,
                      const double* pos, const md_nlist* nl, const double* jac, void* force,
                      double* saved, void* ws, void* ctl, void* stream);

/* Force-matching loss (the mean squared force error over all atoms of all boxes)
 * and its cotangent: L = (1/n) sum_i |F_i - F_ref,i|^2 and G = dL/dF = (2/n)(F - F_ref),
 * the G that md_eam_backward takes.  force: [3][n] as md_eam_forces writes it (float for
 * MD_FP32, double for MD_FP64); f_ref: [3][n] FP64 in the same atom order; loss: one
 * device double; grad_force: [3][n] FP64 or NULL (loss only); ws:
 * md_force_loss_workspace_bytes(n) bytes.  FP64 sums in a fixed order that depends on n
 * alone (bitwise reproducible).  n = 0 writes loss = 0.  MD_ERR_ARG for n < 0 or a NULL
 * loss, ws, force or f_ref (the last two only for n > 0). */
size_t md_force_loss_workspace_bytes(int n_atoms);
int md_force_loss(int n_atoms, md_precision prec, const void* force, const double* f_ref,
                  double* loss, double* grad_force, void* ws, void* stream);

/* Derivative of a loss of the EAM forces of md_eam_forces (Sec. 1.6, eq. 1.6) with
 * respect to the potential's tables -- the hand-written counterpart of the automatic
 * differentiation that gives forces from the network energy in Sec. 2.1 (eq. force).
 * Vector-Jacobian product of the EAM forces with respect to the three spline
 * coefficient vectors: grad_coef[phi | rho | F] += sum_i G_i . dF_i/dc for a
 * cotangent G = dL/dF ([3][n] FP64).  Needs `saved` from md_eam_forces on the
 * same positions and coefficients.  Accumulation is in FP64 and deterministic.
 * grad_coef has phi.ncoef + rho.ncoef + emb.ncoef entries (at most 1024 in all) and is
 * overwritten.  ws: md_backward_workspace_bytes(b, p) bytes.  The accumulation is FP64
 * whatever `prec` the forward pass used. */
size_t md_backward_workspace_bytes(const md_batch* b, const md_eam* p);
int md_eam_backward(const md_batch* b, const md_eam* p, md_precision prec, const double* pos,
                    const md_nlist* nl, const double* saved, const double* grad_force,
                    double* grad_coef, void* ws, void* ctl, void* stream);
/* md_eam_backward for fixed positions whose density Jacobian `jac` (from
 * md_eam_density_jacobian, same positions, list and rho grid) is kept: the F'' term of
 * the rho gradient, sum_i F''_i tau_i jac[i][k], is taken from jac instead of a second
 * visit of every list.  Same arguments, workspace and result (to rounding) otherwise;
 * deterministic.  MD_ERR_ARG for a NULL jac. */
int md_eam_backward_jac(const md_batch* b, const md_eam* p, md_precision prec,
                        const double* pos, const md_nlist* nl, const double* saved,
                        const double* jac, const double* grad_force, double* grad_coef,
                        void* ws, void* ctl, void* stream);

/* ---------------------------------------------------------------------------
 * Behler-Parrinello network potential (Sec. 2.1)
 * ------------------------------------------------------------------------- */

/* E = sum_i E_i (eq. E_as_sum); E_i is a fully connected network (eq. AtomicNN:
 * n_g inputs -> h1 tanh -> h2 tanh -> 1 linear) of the symmetry functions of atom i
 * over its neighbours j within r_cut, f_c(R) = (cos(pi R / r_cut) + 1) / 2:
 *   G2_mu = sum_j exp(-g2_eta[mu] (R_ij - r_s)^2) f_c(R_ij)                       (eq. G2)
 *   G4_mu = 2^(1 - zeta) sum_{j != k} (1 + lambda cos theta_ijk)^zeta
 *           exp(-eta (R_ij^2 + R_ik^2 + R_jk^2)) f_c(R_ij) f_c(R_ik) f_c(R_jk)     (eq. G4)
 * (the radial exponent read as squared; the angular sum over ordered pairs j != k).
 * Forces by eq. force, F_k = -sum_i sum_mu dE_i/dG_mu(i) dG_mu(i)/dR_k, with the
 * network's backward pass and analytic symmetry-function derivatives.  Weights are
 * one device FP64 array: w01 [n_g][h1], b1 [h1], w12 [h1][h2], b2 [h2], w23 [h2], b3,
 * row-major, inputs ordered G2 then G4.  At most MD_BPNN_MAX_G inputs, hidden widths
 * up to MD_BPNN_MAX_HIDDEN, at most 8 distinct G4 eta values and 8 distinct
 * (zeta, lambda) pairs, zeta >= 1, lambda = +-1. */
#define MD_BPNN_MAX_G 64
#define MD_BPNN_MAX_HIDDEN 32
#define MD_BPNN_MAX_NB 128 /* neighbours within r_cut per atom (MD_FLAG_NEIGH_OVERFLOW) */
typedef struct md_bpnn {
  double r_cut, r_s;
  int n_g2, n_g4, h1, h2;
  double g2_eta[MD_BPNN_MAX_G];
  double g4_zeta[MD_BPNN_MAX_G], g4_lambda[MD_BPNN_MAX_G], g4_eta[MD_BPNN_MAX_G];
  const double* weights; /* device */
} md_bpnn;

/* Workspace of md_bpnn_forces: (n_g2 + n_g4 + 1) doubles per atom. */
size_t md_bpnn_workspace_bytes(const md_batch* b, const md_bpnn* p);

/* Energy, forces ([3][n] FP64, overwritten) and virial of the network potential in
 * FP64 from a list built with r_ns >= r_cut; e_atom [n] (optional) receives E_i.
 * The record {E, W[6], K} goes to ev[(step % ev_cap) * n_rep + rep] as in
 * md_lj_forces (W = -sum_i sum (x_j - x_i) (x) dE_i/d(x_j - x_i) over the neighbour
 * vectors each E_i depends on); with vel the trailing half kick is applied and K
 * reduced.  Contributions to a neighbour's force are added with FP64 atomics, so
 * forces can differ from run to run in the last bits (energies and virials are
 * fixed-point and reproducible). */
int md_bpnn_forces(const md_batch* b, const md_bpnn* p, const double* pos, const md_nlist* nl,
                   double* force, double* e_atom, double* vel, double inv_mass, double half_dt,
                   long long* ev, int ev_cap, void* ws, void* ctl, void* stream);

/* ---------------------------------------------------------------------------
 * Analysis (Appendix)
 * ------------------------------------------------------------------------- */

/* Per-atom potential energy and pair virial in FP64 from the current list (valid
 * as for the force passes), for exactly one of eam / lj:
 *   EAM: e_i = F(rhobar_i) + 1/2 sum_j phi(r_ij), evaluated from the B-spline
 *        coefficients; rho_fp[2][n] receives {rhobar_i, F'(rhobar_i)} (required);
 *   LJ:  e_i = 1/2 sum_j U(r_ij) (shifted as in md_lj_forces); rho_fp unused.
 *   w_atom[6][n] = 1/2 sum_j r_ij (x) f_ij (order xx yy zz xy xz yz), r_ij = x_i - x_j,
 *   f_ij the central pair force on i due to j (the Appendix virial read with the pair
 *   force), so sum_i e_i and sum_i w_i are the totals of the force passes' records.
 * Output arrays are [n] / [6][n] FP64 in the current atom order.  Sets
 * MD_FLAG_TABLE_RANGE like the force passes. */
int md_atom_observables(const md_batch* b, const md_eam* eam, const md_lj* lj, const double* pos,
                        const md_nlist* nl, double* e_atom, double* w_atom, double* rho_fp,
                        void* ctl, void* stream);

/* Profiles over n_bins slabs [lo + l width, lo + (l + 1) width) along `axis` of a
 * single box (n_rep = 1; on a periodic axis x is folded into the box first), the
 * statistical definitions of the Appendix for atoms of equal mass (u):
 *   N_l, M_l = N_l m, u_l = sum v / N_l (centre-of-mass velocity),
 *   K_l = sum m (v - u_l) (x) (v - u_l) (eV), T^a_l = K^aa_l / (k_B N_l), T_l = mean,
 *   P_l = (K_l + W_l) / V_l (eV/A^3) with W_l = sum of w_atom over the slab and V_l =
 *   width times the box cross-section, P = trace / 3,
 *   E_pot / M_l = sum e / M_l and E_int / M_l = (sum e + tr K / 2) / M_l (eV/u).
 * out[n_bins][MD_PROF_LEN] (device FP64): N, M, u[3], T^x, T^y, T^z, T,
 * P^{xx yy zz xy xz yz}, P, E_pot/M, E_int/M; empty slabs give zeros.  e_atom and
 * w_atom (md_atom_observables) may be NULL, which zeroes their terms.  Slab sums are
 * accumulated as 64-bit fixed point (2^32 units per eV, angstrom/ps or atom), so the
 * result is reproducible bit for bit; each slab sum must stay within +-2^31 of its
 * unit.  ws: md_profile_workspace_bytes(n_bins) bytes. */
#define MD_PROF_LEN 18
#define MD_MAX_PROFILE_BINS 65536
size_t md_profile_workspace_bytes(int n_bins);
int md_profiles(const md_batch* b, int axis, double lo, double width, int n_bins,
                const double* pos, const double* vel, double mass, const double* e_atom,
                const double* w_atom, double* out, void* ws, void* stream);

/* Copy the control block's sticky flags and counters to host memory
 * host_out[4] = {flags, step, n_rebuilds, max_nneigh} and synchronise the
 * stream.  Returns the md_status of the most severe flag set (MD_OK if none). */
int md_read_flags(const void* ctl, int* host_out, void* stream);

/* Clear the sticky error flags (not the counters). */
int md_clear_flags(void* ctl, void* stream);

/* Kernel timing for measurement harnesses.  md_timer_arm(kernel) makes the next
 * launch of that kernel (on any stream, by this host thread) record a start and a
 * stop event around its execution (hipExtLaunchKernelGGL); md_timer_read waits for
 * the stop event and returns the kernel's duration in milliseconds.  Library-owned
 * events are created on first use.  Not for use under stream capture. */
#define MD_KERNEL_BIN_COUNT 1
#define MD_KERNEL_BUILD 2
#define MD_KERNEL_LJ 3
#define MD_KERNEL_EAM_DENSITY 4
#define MD_KERNEL_EAM_FORCE 5
#define MD_KERNEL_KICK_DRIFT 6
#define MD_KERNEL_EAM_ADJOINT 7
#define MD_KERNEL_BPNN_DESC 8
#define MD_KERNEL_BPNN_FORCE 9
int md_timer_arm(int kernel);
int md_timer_read(float* ms);

/* Human-readable name of a status code (static string). */
const char* md_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* MD950_MD_H */
