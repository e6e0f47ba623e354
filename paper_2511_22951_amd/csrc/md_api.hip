// Set-up entry points of libmd950: planning of cell grids and work tiles, the
// control block, workspace sizes and status reporting.
#include <math.h>
#include <string.h>

#include "md_internal.h"

int md_hip_status(hipError_t e) { return e == hipSuccess ? MD_OK : MD_ERR_HIP; }

namespace {
struct TimerSlot {
  int armed = 0;
  int pending = 0;
  hipEvent_t start = nullptr, stop = nullptr;
};
thread_local TimerSlot g_timer;
}  // namespace

bool md_timer_take(int kernel, hipEvent_t* start, hipEvent_t* stop) {
  if (g_timer.armed == 0 || g_timer.armed != kernel) return false;
  g_timer.armed = 0;
  g_timer.pending = 1;
  *start = g_timer.start;
  *stop = g_timer.stop;
  return true;
}

extern "C" int md_timer_arm(int kernel) {
  if (kernel < MD_KERNEL_BIN_COUNT || kernel > MD_KERNEL_BPNN_FORCE) return MD_ERR_ARG;
  if (!g_timer.start) {
    if (hipEventCreate(&g_timer.start) != hipSuccess) return MD_ERR_HIP;
    if (hipEventCreate(&g_timer.stop) != hipSuccess) return MD_ERR_HIP;
  }
  g_timer.armed = kernel;
  g_timer.pending = 0;
  return MD_OK;
}

extern "C" int md_timer_read(float* ms) {
  if (!ms || !g_timer.pending) return MD_ERR_ARG;
  if (hipEventSynchronize(g_timer.stop) != hipSuccess) return MD_ERR_HIP;
  if (hipEventElapsedTime(ms, g_timer.start, g_timer.stop) != hipSuccess) return MD_ERR_HIP;
  g_timer.pending = 0;
  return MD_OK;
}

static int plan_box(const md_box* bx, double r_ns, int nc[3]) {
  for (int a = 0; a < 3; ++a) {
    const double L = bx->len[a];
    if (!(L > 0.0) || !isfinite(L)) return MD_ERR_BOX;
    // The minimum image of every neighbour must be unique: r_ns < L / 2.
    if (bx->periodic[a] && !(2.0 * r_ns < L)) return MD_ERR_BOX;
    // Cell edge L / nc >= r_ns (Sec. 1.4: grid with cell size R, here rounded so
    // that an integer number of cells tiles the box).
    double q = floor(L / r_ns);
    nc[a] = q < 1.0 ? 1 : (q > 1024.0 ? 1024 : (int)q);
  }
  return MD_OK;
}

extern "C" int md_plan_count(int n_rep, const md_box* boxes, const int* atom_off, double r_ns,
                             int tile_atoms, int* n_cells, int* n_tiles) {
  if (n_rep < 1 || !boxes || !atom_off || !n_cells || !n_tiles) return MD_ERR_ARG;
  if (tile_atoms != MD_TILE || !(r_ns > 0.0)) return MD_ERR_ARG;
  long long cells = 0, tiles = 0;
  if (atom_off[0] != 0) return MD_ERR_ARG;
  for (int r = 0; r < n_rep; ++r) {
    int nc[3];
    int st = plan_box(&boxes[r], r_ns, nc);
    if (st) return st;
    const int na = atom_off[r + 1] - atom_off[r];
    if (na < 0) return MD_ERR_ARG;
    cells += (long long)nc[0] * nc[1] * nc[2];
    tiles += (na + tile_atoms - 1) / tile_atoms;
  }
  if (cells > (1LL << 30) || tiles > (1LL << 30)) return MD_ERR_ARG;
  if (atom_off[n_rep] > MD_MAX_ATOMS) return MD_ERR_ARG;
  *n_cells = (int)cells;
  *n_tiles = (int)tiles;
  return MD_OK;
}

extern "C" int md_plan(int n_rep, const md_box* boxes, const int* atom_off, double r_ns,
                       int tile_atoms, md_domain* domains, md_tile* tiles) {
  int nc_tot, nt_tot;
  int st = md_plan_count(n_rep, boxes, atom_off, r_ns, tile_atoms, &nc_tot, &nt_tot);
  if (st) return st;
  if (!domains || (!tiles && nt_tot > 0)) return MD_ERR_ARG;
  int cell_off = 0, tile_off = 0;
  for (int r = 0; r < n_rep; ++r) {
    md_domain d;
    memset(&d, 0, sizeof(d));
    int nc[3];
    plan_box(&boxes[r], r_ns, nc);
    for (int a = 0; a < 3; ++a) {
      d.lo[a] = boxes[r].lo[a];
      d.len[a] = boxes[r].len[a];
      d.inv_len[a] = 1.0 / boxes[r].len[a];
      d.inv_w[a] = (double)nc[a] / boxes[r].len[a];
      d.nc[a] = nc[a];
      d.periodic[a] = boxes[r].periodic[a] ? 1 : 0;
    }
    d.cell_off = cell_off;
    d.atom_off = atom_off[r];
    d.n_atoms = atom_off[r + 1] - atom_off[r];
    d.tile_off = tile_off;
    d.n_tiles = (d.n_atoms + tile_atoms - 1) / tile_atoms;
    for (int t = 0; t < d.n_tiles; ++t) {
      md_tile& T = tiles[tile_off + t];
      T.rep = r;
      T.first = d.atom_off + t * tile_atoms;
      T.count = d.n_atoms - t * tile_atoms < tile_atoms ? d.n_atoms - t * tile_atoms : tile_atoms;
      T.pad = 0;
    }
    cell_off += nc[0] * nc[1] * nc[2];
    tile_off += d.n_tiles;
    domains[r] = d;
  }
  return MD_OK;
}

extern "C" size_t md_ctl_bytes(void) { return md_align256(sizeof(md_ctl_dev)); }

__global__ void k_ctl_init(md_ctl_dev* ctl) {
  if (threadIdx.x == 0) {
    ctl->rebuild = 0;
    ctl->step = 0;
    ctl->flags = 0;
    ctl->n_rebuilds = 0;
    ctl->max_nneigh = 0;
    ctl->n_dmax = 0;
    ctl->step_next = 0;
    ctl->rec_stale = 1;
    ctl->thr2 = -1.0;
    ctl->pad2 = 0.0;
  }
  for (int k = threadIdx.x; k < MD_DMAX_SLOTS; k += blockDim.x) ctl->dmax[k] = 0.0;
}

__global__ void k_ctl_clear_flags(md_ctl_dev* ctl) {
  if (threadIdx.x == 0) ctl->flags = 0;
}

extern "C" int md_ctl_init(void* ctl, void* stream) {
  if (!ctl) return MD_ERR_ARG;
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(256), 0, (hipStream_t)stream, (md_ctl_dev*)ctl);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" int md_clear_flags(void* ctl, void* stream) {
  if (!ctl) return MD_ERR_ARG;
  hipLaunchKernelGGL(k_ctl_clear_flags, dim3(1), dim3(64), 0, (hipStream_t)stream,
                     (md_ctl_dev*)ctl);
  MD_LAUNCH_CHECK();
  return MD_OK;
}

extern "C" size_t md_workspace_bytes(const md_batch* b) {
  if (!b || b->n_atoms < 0) return 0;
  return md_ws_plan(b).total;
}

extern "C" int md_read_flags(const void* ctl, int* host_out, void* stream) {
  if (!ctl || !host_out) return MD_ERR_ARG;
  md_ctl_dev h;
  hipError_t e = hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e != hipSuccess) return MD_ERR_HIP;
  e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return MD_ERR_HIP;
  host_out[0] = h.flags;
  host_out[1] = h.step;
  host_out[2] = h.n_rebuilds;
  host_out[3] = h.max_nneigh;
  // A void step (a list or carried records used past their validity) comes first: any
  // non-finite position such a step produced is its consequence, not the cause.
  if (h.flags & MD_FLAG_STALE_LIST) return MD_ERR_STALE_LIST;
  if (h.flags & MD_FLAG_STALE_RECORDS) return MD_ERR_STALE_RECORDS;
  if (h.flags & MD_FLAG_NONFINITE) return MD_ERR_NONFINITE;
  if (h.flags & MD_FLAG_NEIGH_OVERFLOW) return MD_ERR_NEIGH_OVERFLOW;
  if (h.flags & MD_FLAG_WALL) return MD_ERR_WALL;
  if (h.flags & MD_FLAG_TABLE_RANGE) return MD_ERR_TABLE_RANGE;
  return MD_OK;
}

extern "C" const char* md_status_string(int s) {
  switch (s) {
    case MD_OK: return "ok";
    case MD_ERR_ARG: return "invalid argument";
    case MD_ERR_BOX: return "box too small for the neighbour radius (need r_ns < L/2 on periodic axes)";
    case MD_ERR_NEIGH_OVERFLOW: return "neighbour list overflow (max_neigh too small)";
    case MD_ERR_TABLE_RANGE: return "potential table evaluated outside its range";
    case MD_ERR_WALL: return "atom outside a non-periodic extent";
    case MD_ERR_NONFINITE: return "non-finite position";
    case MD_ERR_HIP: return "HIP runtime error";
    case MD_ERR_WORKSPACE: return "workspace or capacity too small";
    case MD_ERR_STALE_LIST: return "an atom moved more than half the skin without a list rebuild";
    case MD_ERR_STALE_RECORDS: return "carried FP32 neighbour records declared current after positions changed";
    default: return "unknown status";
  }
}
