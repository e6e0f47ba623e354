"""Python binding of libmd950 (include/md.h).

Argument marshalling only: torch provides device memory and streams, every step
of the MD path runs in the library's HIP kernels.  Function names follow the C
entry points (md_bin_cells, md_build_neighbors, md_lj_forces, md_eam_forces,
md_verlet_step, md_eam_backward); the small classes below hold the buffers
those calls take.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _native as N
from ._native import MDError, check  # noqa: F401

ACCEL = 9648.5332157  # 1 eV/(u angstrom) in angstrom/ps^2 (unit conversion for callers)


def ev_buffer(ev_cap, n_rep, device="cuda"):
    """Per-step records [ev_cap, n_rep, 8] (int64 fixed point, md.h MD_EV_SCALE)."""
    return torch.zeros((ev_cap, n_rep, N.MD_EV_LEN), dtype=torch.int64, device=device)


def ev_values(ev):
    """Records in eV: {E_pot, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz, K} as float64 numpy."""
    return ev.cpu().numpy().astype(np.float64) / N.MD_EV_SCALE


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _require_cuda(device):
    if torch.device(device).type != "cuda":
        raise RuntimeError("the MD path runs on the GPU only (device %s)" % device)
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the MD path has no CPU fallback")


# ----------------------------------------------------------------------------
# Plans (cell grids and work tiles of one box or a batch of boxes)
# ----------------------------------------------------------------------------
def _cbox(box):
    b = N.Box()
    for a in range(3):
        b.lo[a] = float(box.lo[a])
        b.len[a] = float(box.len[a])
        b.periodic[a] = int(box.periodic[a])
    return b


class Plan:
    """md_plan for n_rep boxes with atom_counts atoms each, uploaded to the device."""

    def __init__(self, boxes, atom_counts, r_ns, device="cuda"):
        _require_cuda(device)
        L = N.lib()
        n_rep = len(boxes)
        cb = (N.Box * n_rep)(*[_cbox(b) for b in boxes])
        off = np.zeros(n_rep + 1, np.int32)
        off[1:] = np.cumsum(np.asarray(atom_counts, np.int64))
        coff = (C.c_int * (n_rep + 1))(*off.tolist())
        nc, nt = C.c_int(), C.c_int()
        check(L.md_plan_count(n_rep, cb, coff, float(r_ns), N.MD_TILE, C.byref(nc), C.byref(nt)),
              "md_plan_count")
        doms = (N.Domain * n_rep)()
        tiles = (N.Tile * max(1, nt.value))()
        check(L.md_plan(n_rep, cb, coff, float(r_ns), N.MD_TILE, doms, tiles), "md_plan")
        self.host_domains = doms
        self.host_tiles = tiles
        self.atom_off = off
        self.n_rep, self.n_atoms = n_rep, int(off[-1])
        self.n_cells, self.n_tiles = nc.value, nt.value
        self.r_ns = float(r_ns)
        self.device = torch.device(device)
        self.d_domains = torch.from_numpy(
            np.frombuffer(bytes(doms), np.uint8).copy()).to(self.device)
        self.d_tiles = torch.from_numpy(np.frombuffer(bytes(tiles), np.uint8).copy()).to(self.device)
        self.c = N.Batch(n_rep, self.n_atoms, self.n_cells, self.n_tiles, N.MD_TILE, 0, self.r_ns,
                         self.d_domains.data_ptr(), self.d_tiles.data_ptr())
        self.cells_per_axis = [tuple(doms[r].nc) for r in range(n_rep)]

    def workspace_bytes(self):
        return int(N.lib().md_workspace_bytes(C.byref(self.c)))


# ----------------------------------------------------------------------------
# Neighbour list
# ----------------------------------------------------------------------------
class NeighborList:
    """Padded strided ELL list (md_nlist) for `lanes` lanes per atom."""

    def __init__(self, n_atoms, max_neigh=128, lanes=4, device="cuda", block=0):
        """block: threads per workgroup of the force passes (0: the library default, 1024)."""
        if max_neigh % lanes:
            max_neigh += lanes - max_neigh % lanes
        self.n, self.max_neigh, self.lanes, self.block = n_atoms, max_neigh, lanes, int(block)
        self.npad = (n_atoms + 63) // 64 * 64
        self.neigh = torch.zeros(max_neigh * self.npad, dtype=torch.int32, device=device)
        self.nneigh = torch.zeros(max(1, n_atoms), dtype=torch.int32, device=device)
        self.c = N.NList(self.neigh.data_ptr(), self.nneigh.data_ptr(), max_neigh, lanes,
                         self.block)

    def set_block(self, block):
        """Change the force passes' workgroup size (a launch-shape choice)."""
        self.block = int(block)
        self.c.block = self.block

    def lengths(self):
        """List lengths (the image flag masked off)."""
        return self.nneigh[:self.n] & (N.MD_NN_IMG - 1)

    def host_lists(self):
        """Per atom (current order) the array of neighbour indices (current order)."""
        nn = self.nneigh.cpu().numpy()[:self.n] & (N.MD_NN_IMG - 1)
        raw = self.neigh.cpu().numpy().reshape(self.max_neigh // self.lanes, self.npad, self.lanes)
        out = []
        for i in range(self.n):
            k = np.arange(nn[i])
            out.append(raw[k // self.lanes, i, k % self.lanes].copy())
        return out


# ----------------------------------------------------------------------------
# Atom state
# ----------------------------------------------------------------------------
class State:
    """Device arrays of one batch: pos [n,4] (double4), vel/force/pos_ref [3,n], id [n],
    cell_start, workspace and the control block."""

    def __init__(self, plan: Plan, pos, vel, precision=N.MD_FP64, ids=None):
        dev = plan.device
        n = plan.n_atoms
        pos = np.asarray(pos, np.float64).reshape(n, 3)
        vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, np.float64).reshape(n, 3)
        p4 = np.zeros((n, 4))
        p4[:, :3] = pos
        self.plan = plan
        self.n = n
        self.precision = precision
        self.pos = torch.from_numpy(p4).to(dev)
        self.vel = torch.from_numpy(np.ascontiguousarray(vel.T)).to(dev)
        fdt = torch.float32 if precision == N.MD_FP32 else torch.float64
        self.force = torch.zeros((3, n), dtype=fdt, device=dev)
        ids = np.arange(n, dtype=np.int32) if ids is None else np.asarray(ids, np.int32)
        self.id = torch.from_numpy(ids.copy()).to(dev)
        self.pos_ref = torch.zeros((3, n), dtype=torch.float64, device=dev)
        self.cell_start = torch.zeros(plan.n_cells + 1, dtype=torch.int32, device=dev)
        self.ws = torch.zeros(max(256, plan.workspace_bytes()), dtype=torch.uint8, device=dev)
        self.ctl = torch.zeros(int(N.lib().md_ctl_bytes()), dtype=torch.uint8, device=dev)
        check(N.lib().md_ctl_init(_ptr(self.ctl), _stream()), "md_ctl_init")

    # host views, ordered by original id
    def _order(self):
        return np.argsort(self.id.cpu().numpy(), kind="stable")

    def positions(self):
        return self.pos[:, :3].cpu().numpy()[self._order()]

    def velocities(self):
        return self.vel.t().cpu().numpy()[self._order()]

    def forces(self):
        return self.force.t().double().cpu().numpy()[self._order()]

    def read_flags(self):
        out = (C.c_int * 4)()
        st = N.lib().md_read_flags(_ptr(self.ctl), out, _stream())
        return st, {"flags": out[0], "step": out[1], "n_rebuilds": out[2], "max_nneigh": out[3]}

    def check_flags(self, what="device flags"):
        st, info = self.read_flags()
        check(st, what)
        return info

    def clear_flags(self):
        check(N.lib().md_clear_flags(_ptr(self.ctl), _stream()), "md_clear_flags")


# ----------------------------------------------------------------------------
# Potentials
# ----------------------------------------------------------------------------
def md_spline_fit(y, h, dy_lo, dy_hi, device="cuda"):
    """Complete cubic spline fit on the device; returns K + 2 coefficients."""
    y = torch.as_tensor(np.asarray(y, np.float64), device=device)
    coef = torch.zeros(y.shape[0] + 2, dtype=torch.float64, device=device)
    check(N.lib().md_spline_fit(_ptr(y), int(y.shape[0]), float(h), float(dy_lo), float(dy_hi),
                                _ptr(coef), _stream()), "md_spline_fit")
    return coef


class EAMPotential:
    """Device B-spline coefficients of phi, rho, F and the packed interval tables."""

    def __init__(self, c_phi, c_rho, c_emb, r_lo, r_h, e_lo, e_h, r_cut, device="cuda"):
        dev = torch.device(device)
        parts = [torch.as_tensor(np.asarray(c, np.float64) if not torch.is_tensor(c) else c,
                                 dtype=torch.float64, device=dev).reshape(-1)
                 for c in (c_phi, c_rho, c_emb)]
        # one buffer (phi | rho | F), so that a new coefficient vector is one copy
        self._flat = torch.cat(parts).contiguous()
        n0, n1 = parts[0].shape[0], parts[1].shape[0]
        self.coef = [self._flat[:n0], self._flat[n0:n0 + n1], self._flat[n0 + n1:]]
        self.r_lo, self.r_h, self.e_lo, self.e_h = float(r_lo), float(r_h), float(e_lo), float(e_h)
        self.r_cut = float(r_cut)
        self.device = dev
        self._tables = {}
        self.version = 0  # advanced by every coefficient change
        self._build_struct()

    def _build_struct(self):
        cp, cr, ce = self.coef
        self.c = N.EAM(N.Spline(cp.data_ptr(), cp.shape[0], 0, self.r_lo, self.r_h),
                       N.Spline(cr.data_ptr(), cr.shape[0], 0, self.r_lo, self.r_h),
                       N.Spline(ce.data_ptr(), ce.shape[0], 0, self.e_lo, self.e_h), self.r_cut)

    @classmethod
    def from_table(cls, table, device="cuda"):
        """Fit a tabulated EAM (values on a grid plus end slopes) on the device."""
        fits = [md_spline_fit(tf.y, tf.h, tf.dy_lo, tf.dy_hi, device)
                for tf in (table.phi, table.rho, table.emb)]
        if table.phi.x_lo != table.rho.x_lo or table.phi.h != table.rho.h:
            raise ValueError("phi and rho must share one grid")
        return cls(*fits, table.rho.x_lo, table.rho.h, table.emb.x_lo, table.emb.h, table.r_cut,
                   device)

    def set_coefficients(self, c_phi=None, c_rho=None, c_emb=None):
        for k, c in enumerate((c_phi, c_rho, c_emb)):
            if c is not None:
                self.coef[k].copy_(torch.as_tensor(c, dtype=torch.float64))
        self.version += 1

    def set_coefficients_flat(self, c):
        """All coefficients at once from one (phi | rho | F) vector."""
        self._flat.copy_(torch.as_tensor(c, dtype=torch.float64).reshape(-1))
        self.version += 1

    def coefficients_flat(self):
        """A copy of the (phi | rho | F) coefficient vector."""
        return self._flat.clone()

    def table(self, precision):
        """Packed interval tables (md_eam_prepare), prepared from the current coefficients on
        every call (the buffer is kept: its size depends on the grids alone)."""
        if precision not in self._tables:
            nbytes = int(N.lib().md_eam_table_bytes(C.byref(self.c), precision))
            if nbytes == 0:
                raise ValueError("invalid EAM description")
            t = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
            self._tables[precision] = t
        t = self._tables[precision]
        check(N.lib().md_eam_prepare(C.byref(self.c), precision, _ptr(t), _stream()),
              "md_eam_prepare")
        return t


def lj_params(eps, sigma, r_cut):
    return N.LJ(float(eps), float(sigma), float(r_cut))


def walls_params(walls):
    if not walls:
        return None
    return N.Walls(1, int(walls["axis"]), float(walls["piston_z0"]), float(walls["piston_v"]),
                   float(walls["top_z"]))


# ----------------------------------------------------------------------------
# The C entry points
# ----------------------------------------------------------------------------
def md_bin_cells(st: State, mode=N.MD_ALWAYS, stream=None):
    check(N.lib().md_bin_cells(C.byref(st.plan.c), mode, _ptr(st.pos), _ptr(st.vel), _ptr(st.id),
                               _ptr(st.pos_ref), _ptr(st.cell_start), _ptr(st.ws), _ptr(st.ctl),
                               _stream(stream)), "md_bin_cells")


def md_build_neighbors(st: State, nl: NeighborList, mode=N.MD_ALWAYS, stream=None):
    check(N.lib().md_build_neighbors(C.byref(st.plan.c), mode, _ptr(st.pos), _ptr(st.cell_start),
                                     C.byref(nl.c), _ptr(st.ctl), _stream(stream)),
          "md_build_neighbors")


def md_lj_forces(st: State, p, nl: NeighborList, inv_mass=0.0, half_dt=0.0, kick=False,
                 ev=None, ev_cap=1, drift=None, stream=None):
    vel = st.vel if kick else None
    check(N.lib().md_lj_forces(C.byref(st.plan.c), C.byref(p), st.precision, _ptr(st.pos),
                               C.byref(nl.c), _ptr(st.force), _ptr(vel), float(inv_mass),
                               float(half_dt), C.byref(drift) if drift is not None else None,
                               _ptr(ev), int(ev_cap), _ptr(st.ws), _ptr(st.ctl),
                               _stream(stream)), "md_lj_forces")


def drift_params(pos_out, pos_ref, dt, half_skin, walls=None, rec_in=None, rec_out=None,
                 rec_current=False, langevin=None):
    """md_drift: the next step's kick-drift to fuse into md_lj_forces or md_eam_forces;
    rec_in / rec_out: FP32 neighbour records carried from step to step (uint8 [16 n]
    device tensors, or None); rec_current: rec_in is known to be current (no launch to
    check it; a wrong claim raises MD_ERR_STALE_RECORDS); langevin: an N.Langevin
    (langevin_params) for the Langevin update before the next half kick, which the caller
    keeps alive while the md_drift is in use."""
    w = walls_params(walls) if isinstance(walls, dict) else walls
    return N.Drift(_ptr(pos_out), _ptr(pos_ref), float(dt), float(half_skin),
                   w if w is not None else N.Walls(0, 2, 0.0, 0.0, 0.0), _ptr(rec_in),
                   _ptr(rec_out), int(bool(rec_current)), 0,
                   C.addressof(langevin) if langevin is not None else None)


def md_eam_forces(st: State, pot: EAMPotential, nl: NeighborList, table=None, saved=None,
                  inv_mass=0.0, half_dt=0.0, kick=False, ev=None, ev_cap=1, drift=None,
                  stream=None):
    table = pot.table(st.precision) if table is None else table
    vel = st.vel if kick else None
    check(N.lib().md_eam_forces(C.byref(st.plan.c), C.byref(pot.c), st.precision, _ptr(table),
                                _ptr(st.pos), C.byref(nl.c), _ptr(st.force), _ptr(saved),
                                _ptr(vel), float(inv_mass), float(half_dt),
                                C.byref(drift) if drift is not None else None, _ptr(ev),
                                int(ev_cap), _ptr(st.ws), _ptr(st.ctl), _stream(stream)),
          "md_eam_forces")


def md_eam_forces_jac(st: State, pot: EAMPotential, nl: NeighborList, jac, table=None,
                      saved=None, stream=None):
    """Forces of fixed positions with the density from the kept density Jacobian jac
    ([n, n_rho] FP64, md_eam_density_jacobian of the same positions and list)."""
    table = pot.table(st.precision) if table is None else table
    n_rho = pot.coef[1].shape[0]
    if jac.dtype != torch.float64 or tuple(jac.shape) != (st.plan.n_atoms, n_rho) or \
            not jac.is_contiguous():
        raise ValueError("jac must be a contiguous [n, n_rho] float64 tensor")
    check(N.lib().md_eam_forces_jac(C.byref(st.plan.c), C.byref(pot.c), st.precision, _ptr(table),
                                    _ptr(st.pos), C.byref(nl.c), _ptr(jac), _ptr(st.force),
                                    _ptr(saved), _ptr(st.ws), _ptr(st.ctl), _stream(stream)),
          "md_eam_forces_jac")


def md_eam_forces_noalloc(st: State, pot: EAMPotential, nl: NeighborList, table=None,
                          saved=None, inv_mass=0.0, half_dt=0.0, kick=False, ev=None, ev_cap=1,
                          drift=None, stream=None):
    """md_eam_forces with the library's static scratch instead of the state's workspace."""
    table = pot.table(st.precision) if table is None else table
    vel = st.vel if kick else None
    check(N.lib().md_eam_forces_noalloc(C.byref(st.plan.c), C.byref(pot.c), st.precision,
                                        _ptr(table), _ptr(st.pos), C.byref(nl.c), _ptr(st.force),
                                        _ptr(saved), _ptr(vel), float(inv_mass), float(half_dt),
                                        C.byref(drift) if drift is not None else None, _ptr(ev),
                                        int(ev_cap), _ptr(st.ctl), _stream(stream)),
          "md_eam_forces_noalloc")


def langevin_params(st: State, thermostat):
    """md_langevin from {"seed": int, "axis": 0-2, "regions": [{"lo", "hi", "T", "gamma",
    "u": (ux, uy, uz)}, ...]} (lo/hi default to an unbounded slab, u to zero)."""
    if thermostat is None or isinstance(thermostat, N.Langevin):
        return thermostat
    regs = thermostat["regions"]
    if not 1 <= len(regs) <= N.MD_MAX_THERMO_REGIONS:
        raise ValueError("1 to %d thermostat regions" % N.MD_MAX_THERMO_REGIONS)
    lg = N.Langevin()
    lg.id = _ptr(st.id)
    lg.seed = int(thermostat.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    lg.axis = int(thermostat.get("axis", 2))
    lg.n_regions = len(regs)
    for q, r in enumerate(regs):
        g = lg.region[q]
        g.lo = float(r.get("lo", -math.inf))
        g.hi = float(r.get("hi", math.inf))
        g.temperature = float(r["T"])
        g.gamma = float(r["gamma"])
        for k, x in enumerate(r.get("u", (0.0, 0.0, 0.0))):
            g.u[k] = float(x)
    return lg


def md_verlet_step(st: State, phase, dt, inv_mass, walls=None, half_skin=-1.0, langevin=None,
                   stream=None):
    w = walls_params(walls) if isinstance(walls, dict) else walls
    lg = langevin_params(st, langevin)
    check(N.lib().md_verlet_step(C.byref(st.plan.c), phase, float(dt), _ptr(st.pos), _ptr(st.vel),
                                 _ptr(st.force), st.precision, float(inv_mass),
                                 C.byref(w) if w is not None else None,
                                 C.byref(lg) if lg is not None else None, _ptr(st.pos_ref),
                                 float(half_skin), _ptr(st.ctl), _stream(stream)),
          "md_verlet_step")


class BPNNPotential:
    """md_bpnn: symmetry-function parameters by value and the network weights on the
    device ({"r_cut", "r_s", "g2_eta", "g4_zeta", "g4_lambda", "g4_eta", "w01", "b1",
    "w12", "b2", "w23", "b3"})."""

    def __init__(self, params, device="cuda"):
        w01 = np.asarray(params["w01"], np.float64)
        ng, h1 = w01.shape
        w12 = np.asarray(params["w12"], np.float64)
        h2 = w12.shape[1]
        n2, n4 = len(params["g2_eta"]), len(params["g4_eta"])
        if n2 + n4 != ng or w12.shape[0] != h1:
            raise ValueError("network shapes do not match the symmetry functions")
        flat = np.concatenate([w01.ravel(), np.asarray(params["b1"], np.float64).ravel(),
                               w12.ravel(), np.asarray(params["b2"], np.float64).ravel(),
                               np.asarray(params["w23"], np.float64).ravel(),
                               np.atleast_1d(np.asarray(params["b3"], np.float64))])
        self.weights = torch.from_numpy(flat).to(device)
        c = N.BPNN()
        c.r_cut, c.r_s = float(params["r_cut"]), float(params["r_s"])
        c.n_g2, c.n_g4, c.h1, c.h2 = n2, n4, h1, h2
        for k in range(n2):
            c.g2_eta[k] = float(params["g2_eta"][k])
        for k in range(n4):
            c.g4_zeta[k] = float(params["g4_zeta"][k])
            c.g4_lambda[k] = float(params["g4_lambda"][k])
            c.g4_eta[k] = float(params["g4_eta"][k])
        c.weights = self.weights.data_ptr()
        self.c = c
        self.r_cut = c.r_cut


def md_bpnn_forces(st: State, pot: BPNNPotential, nl: NeighborList, inv_mass=0.0, half_dt=0.0,
                   kick=False, ev=None, ev_cap=1, e_atom=None, ws=None, stream=None):
    """Network-potential forces into st.force (FP64); ws: md_bpnn_workspace_bytes bytes."""
    if st.force.dtype != torch.float64:
        raise ValueError("the network potential computes FP64 forces")
    if ws is None:
        ws = torch.empty(max(256, int(N.lib().md_bpnn_workspace_bytes(C.byref(st.plan.c),
                                                                         C.byref(pot.c)))),
                         dtype=torch.uint8, device=st.pos.device)
    vel = st.vel if kick else None
    check(N.lib().md_bpnn_forces(C.byref(st.plan.c), C.byref(pot.c), _ptr(st.pos), C.byref(nl.c),
                                 _ptr(st.force), _ptr(e_atom), _ptr(vel), float(inv_mass),
                                 float(half_dt), _ptr(ev), int(ev_cap), _ptr(ws), _ptr(st.ctl),
                                 _stream(stream)), "md_bpnn_forces")
    return ws


def md_atom_observables(st: State, nl: NeighborList, eam: EAMPotential = None, lj=None,
                        stream=None):
    """Per-atom energy [n], pair virial [6, n] and, for EAM, {rhobar, F'} [2, n] (FP64,
    current atom order) from the current list."""
    dev = st.pos.device
    n = st.n
    e = torch.empty(n, dtype=torch.float64, device=dev)
    w = torch.empty((6, n), dtype=torch.float64, device=dev)
    rf = torch.empty((2, n), dtype=torch.float64, device=dev) if eam is not None else None
    check(N.lib().md_atom_observables(C.byref(st.plan.c),
                                      C.byref(eam.c) if eam is not None else None,
                                      C.byref(lj) if lj is not None else None, _ptr(st.pos),
                                      C.byref(nl.c), _ptr(e), _ptr(w), _ptr(rf), _ptr(st.ctl),
                                      _stream(stream)), "md_atom_observables")
    return e, w, rf


def md_profiles(st: State, axis, lo, width, n_bins, mass, e_atom=None, w_atom=None, ws=None,
                stream=None):
    """Slab profiles [n_bins, MD_PROF_LEN] (fields N.PROF_FIELDS) of a single box."""
    dev = st.pos.device
    out = torch.empty((n_bins, N.MD_PROF_LEN), dtype=torch.float64, device=dev)
    if ws is None:
        ws = torch.empty(max(256, int(N.lib().md_profile_workspace_bytes(int(n_bins)))),
                         dtype=torch.uint8, device=dev)
    check(N.lib().md_profiles(C.byref(st.plan.c), int(axis), float(lo), float(width),
                              int(n_bins), _ptr(st.pos), _ptr(st.vel), float(mass),
                              _ptr(e_atom), _ptr(w_atom), _ptr(out), _ptr(ws), _stream(stream)),
          "md_profiles")
    return out


def md_force_loss(force, f_ref, precision, grad_force=None, ws=None, stream=None):
    """L = (1/n) sum |F - F_ref|^2 over the n atoms of force ([3, n], float for MD_FP32, double
    for MD_FP64) and f_ref ([3, n] FP64); writes G = (2/n)(F - F_ref) into grad_force ([3, n]
    FP64) when given.  Returns L as a 0-dim device tensor."""
    L = N.lib()
    _require_cuda(f_ref.device)
    fdt = torch.float32 if precision == N.MD_FP32 else torch.float64
    if f_ref.dtype != torch.float64 or f_ref.dim() != 2 or f_ref.shape[0] != 3 or \
            not f_ref.is_contiguous():
        raise ValueError("f_ref must be a contiguous [3, n] float64 tensor")
    if force.dtype != fdt or force.shape != f_ref.shape or not force.is_contiguous() or \
            force.device != f_ref.device:
        raise ValueError("force must be a contiguous [3, n] %s tensor" % fdt)
    if grad_force is not None and (grad_force.dtype != torch.float64 or
                                   grad_force.shape != f_ref.shape or
                                   not grad_force.is_contiguous() or
                                   grad_force.device != f_ref.device):
        raise ValueError("grad_force must be a contiguous [3, n] float64 tensor")
    n = int(f_ref.shape[1])
    nb = int(L.md_force_loss_workspace_bytes(n))
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=f_ref.device)
    loss = torch.empty((), dtype=torch.float64, device=f_ref.device)
    check(L.md_force_loss(n, int(precision), _ptr(force), _ptr(f_ref), _ptr(loss),
                          _ptr(grad_force), _ptr(ws), _stream(stream)), "md_force_loss")
    return loss


def md_eam_density_jacobian(st: State, pot: EAMPotential, nl: NeighborList, out=None,
                            stream=None):
    """d rhobar_i / d c_rho_k of the current positions as an [n, n_rho] FP64 tensor."""
    L = N.lib()
    n, n_rho = st.plan.n_atoms, pot.coef[1].shape[0]
    nb = int(L.md_density_jacobian_bytes(C.byref(st.plan.c), C.byref(pot.c)))
    if nb == 0 and n > 0:
        raise ValueError("density Jacobian not available for %d rho coefficients" % n_rho)
    if out is None:
        out = torch.empty((n, n_rho), dtype=torch.float64, device=st.pos.device)
    elif out.dtype != torch.float64 or tuple(out.shape) != (n, n_rho) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [%d, %d] float64 tensor" % (n, n_rho))
    check(L.md_eam_density_jacobian(C.byref(st.plan.c), C.byref(pot.c), _ptr(st.pos),
                                    C.byref(nl.c), _ptr(out), _ptr(st.ctl), _stream(stream)),
          "md_eam_density_jacobian")
    return out


def md_eam_backward(st: State, pot: EAMPotential, nl: NeighborList, saved, grad_force, ws=None,
                    stream=None, jac=None):
    """grad_force: [3, n] FP64 cotangent in the current atom order.  Returns [n_coef total].
    jac: the density Jacobian of the same positions (md_eam_density_jacobian), if kept."""
    L = N.lib()
    nb = int(L.md_backward_workspace_bytes(C.byref(st.plan.c), C.byref(pot.c)))
    if nb == 0:
        raise ValueError("backward not available for this spline size")
    if ws is None or ws.numel() < nb:
        ws = torch.zeros(nb, dtype=torch.uint8, device=st.pos.device)
    out = torch.empty(sum(c.shape[0] for c in pot.coef), dtype=torch.float64, device=st.pos.device)
    if jac is None:
        check(L.md_eam_backward(C.byref(st.plan.c), C.byref(pot.c), st.precision, _ptr(st.pos),
                                C.byref(nl.c), _ptr(saved), _ptr(grad_force), _ptr(out),
                                _ptr(ws), _ptr(st.ctl), _stream(stream)), "md_eam_backward")
    else:
        check(L.md_eam_backward_jac(C.byref(st.plan.c), C.byref(pot.c), st.precision,
                                    _ptr(st.pos), C.byref(nl.c), _ptr(saved), _ptr(jac),
                                    _ptr(grad_force), _ptr(out), _ptr(ws), _ptr(st.ctl),
                                    _stream(stream)), "md_eam_backward_jac")
    return out
