"""NVE driver: the sequence of library calls that makes one velocity-Verlet step
(Sec. 1.5) with neighbour-list rebuilds (Sec. 1.4), optionally captured once into
a HIP graph and replayed.

One step, all on one stream, no host synchronisation:
  md_verlet_step(KICK_DRIFT)          v += dt/2 f/m; x += dt v; walls; displacements
  md_bin_cells, md_build_neighbors    rebuild (policy below)
  md_eam_forces / md_lj_forces        forces, energy, virial, trailing kick v += dt/2 f/m

With fused=True (EAM or LJ) the force pass also performs the next step's kick-drift
(md_drift), writing the new positions into a second buffer that becomes current
after the call, so from the second step on a step is rebuild + density + force.
The arithmetic is the same, bit for bit; between steps the state is then one
kick-drift ahead: positions x(n + 1), velocities v(n + 1/2) (`previous_positions`
returns x(n)).

With a thermostat ({"seed", "axis", "regions": [{"lo", "hi", "T", "gamma", "u"}]}) the
kick-drift starts with the Langevin velocity update of md_langevin (NVT, Sec. 1.5), in
the separate kick-drift or in the fused one (md_drift.langevin) alike.

Rebuild policies (both in the paper):
  rebuild_every = 0: on the threshold (Sec. 1.4) -- the rebuild kernels run every
      step in MD_IF_FLAGGED mode and do work only when an atom moved > skin/2;
  rebuild_every = k: every k steps (the benchmark of Sec. 1.7) -- the rebuild
      kernels are launched only on those steps; the force pass verifies the
      half-skin criterion on every step (MD_ERR_STALE_LIST if violated), so a run
      that ends with clear flags used valid lists throughout.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _native as N
from . import md


def graph_period(rebuild_every, fused):
    """Steps after which a captured step sequence repeats exactly: the rebuild period k
    (rebuilds on the steps n with (n + 1) % k == 0), times 2 in fused mode when k is odd
    (the two position buffers trade places every step)."""
    k = max(1, int(rebuild_every))
    return 2 * k // math.gcd(2, k) if fused else k


def timed_graph_plan(n_steps, rebuild_every, fused, graph_steps):
    """How a run of exactly n_steps steps, starting at a multiple of the graph period, is
    made of graph replays only: q replays of a main graph of G steps (a multiple of the
    period near graph_steps, at most n_steps) and, if r = n_steps - q G > 0, one replay of a
    tail graph of r steps.  Returns (G, q, r)."""
    n_steps = int(n_steps)
    if n_steps < 0:
        raise ValueError("negative step count")
    P = graph_period(rebuild_every, fused)
    G = P * max(1, min(int(graph_steps), n_steps) // P)
    if G > n_steps:  # shorter than one period: the tail graph alone
        return G, 0, n_steps
    return G, n_steps // G, n_steps % G


def fused_grid_fits(n_tiles, lanes, block=0):
    """Whether a force pass of `lanes` lanes per atom over n_tiles tiles (block / (64 lanes)
    tiles per block of `block` threads, default 1024; the grid rounded up to a multiple of 8)
    fits the displacement slots the fused kick-drift publishes into."""
    tpb = max(1, (block or 1024) // (64 * lanes))
    blocks = (n_tiles + tpb - 1) // tpb
    return (blocks + 7) // 8 * 8 <= N.MD_DRIFT_MAX_BLOCKS


class Simulation:
    def __init__(self, system, precision=N.MD_FP64, lanes=4, max_neigh=128, ev_cap=1024,
                 device="cuda", table=None, rebuild_every=0, fused=False, thermostat=None,
                 block=0, carry_records=True):
        """carry_records: in fused FP32 runs with fixed-period rebuilds, the fused kick-drift
        writes the next step's neighbour records (md_drift.rec_out) and the next force call
        takes them (rec_in) instead of converting the positions again, with no conversion
        launch between rebuilds; False (and threshold rebuilds, where the device decides
        whether the atoms are reordered) converts every step."""
        self.sys = system
        self.fused = bool(fused) and system.potential in ("eam", "lj")
        self.primed = False  # fused: the last force pass already did the next kick-drift
        self.pos_alt = None
        self.carry = bool(carry_records) and self.fused and precision == N.MD_FP32
        self.rec = self.rec_alt = None  # carried FP32 records of pos and of pos_alt
        self.rec_fresh = False  # self.rec holds the records of the current positions
        self.rebuild_every = int(rebuild_every)
        self.n_steps = 0
        self.precision = precision
        if system.potential == "lj":
            r_cut = system.lj.r_cut
        elif system.potential == "bpnn":
            r_cut = system.extra["bpnn"]["r_cut"]
        else:
            r_cut = system.eam.r_cut
        self.r_ns = r_cut + system.skin
        self.plan = md.Plan([system.box], [system.pos.shape[0]], self.r_ns, device)
        self.state = md.State(self.plan, system.pos, system.vel, precision)
        self.nl = md.NeighborList(self.plan.n_atoms, max_neigh, lanes, device, block=block)
        if self.fused and not fused_grid_fits(self.plan.n_tiles, lanes, block):
            raise ValueError("fused kick-drift: %d lanes per atom over %d atoms exceed the "
                             "force pass's %d displacement slots; use fewer lanes or fused=False"
                             % (lanes, self.plan.n_atoms, N.MD_DRIFT_MAX_BLOCKS))
        self.inv_mass = 1.0 / system.mass
        self.dt = system.dt_ps
        self.half_skin = 0.5 * system.skin
        self.walls = md.walls_params(system.walls)
        self.langevin = md.langevin_params(self.state, thermostat)
        self.ev_cap = ev_cap
        self.ev = md.ev_buffer(ev_cap, 1, device)
        self.bpnn = None
        if system.potential == "lj":
            self.lj = md.lj_params(system.lj.eps, system.lj.sigma, system.lj.r_cut)
            self.pot = None
        elif system.potential == "bpnn":
            if precision != N.MD_FP64:
                raise ValueError("the network potential runs in FP64")
            self.bpnn = md.BPNNPotential(system.extra["bpnn"], device)
            self.bpnn_ws = None
            self.pot = None
        else:
            self.pot = md.EAMPotential.from_table(table or system.table, device)
            self.table = self.pot.table(precision)
        self.graph = None
        self.graph_steps = 0
        self.eager_steps = 0  # steps launched outside graph capture (timed-region checks)
        self._capturing = False

    # -- pieces ---------------------------------------------------------------
    def forces(self, kick, ev=True):
        st = self.state
        half_dt = 0.5 * self.dt if kick else 0.0
        evb = self.ev if ev else None
        if self.bpnn is not None:
            self.bpnn_ws = md.md_bpnn_forces(st, self.bpnn, self.nl, self.inv_mass, half_dt,
                                             kick=True, ev=evb, ev_cap=self.ev_cap,
                                             ws=self.bpnn_ws)
        elif self.pot is None:
            md.md_lj_forces(st, self.lj, self.nl, self.inv_mass, half_dt, kick=True, ev=evb,
                            ev_cap=self.ev_cap)
        else:
            md.md_eam_forces(st, self.pot, self.nl, self.table, None, self.inv_mass, half_dt,
                             kick=True, ev=evb, ev_cap=self.ev_cap)

    def setup(self):
        """Initial binning, list and forces (step 0: energies with the initial velocities)."""
        md.md_bin_cells(self.state, N.MD_ALWAYS)
        md.md_build_neighbors(self.state, self.nl, N.MD_ALWAYS)
        self.forces(kick=False)
        return self

    def rebuild(self):
        """Rebuild the cell order and the list now (e.g. when switching rebuild policy)."""
        self.rec_fresh = False
        md.md_bin_cells(self.state, N.MD_ALWAYS)
        md.md_build_neighbors(self.state, self.nl, N.MD_ALWAYS)

    def set_rebuild_every(self, k):
        """Switch the rebuild policy; rebuilds now so that the next period starts fresh."""
        self.rebuild_every = int(k)
        self.graph = None
        self.rebuild()
        if k > 0:
            self.n_steps -= self.n_steps % k

    def step(self, ev=True):
        st = self.state
        if not self.primed:
            self.rec_fresh = False
            md.md_verlet_step(st, N.MD_KICK_DRIFT, self.dt, self.inv_mass, self.walls,
                              self.half_skin, langevin=self.langevin)
        k = self.rebuild_every
        if k <= 0:
            self.rec_fresh = False  # the device decides whether the atoms are reordered
            md.md_bin_cells(st, N.MD_IF_FLAGGED)
            md.md_build_neighbors(st, self.nl, N.MD_IF_FLAGGED)
        elif (self.n_steps + 1) % k == 0:
            self.rec_fresh = False
            md.md_bin_cells(st, N.MD_ALWAYS)
            md.md_build_neighbors(st, self.nl, N.MD_ALWAYS)
        if self.fused:
            if self.pos_alt is None:
                self.pos_alt = torch.empty_like(st.pos)
            carry = self.carry and self.rebuild_every > 0
            if not carry:
                self.rec_fresh = False
            elif self.rec is None:
                # contents need not be valid: md_ctl_init and the first kick-drift mark the
                # positions as changed, so the first force call converts them
                self.rec = torch.empty(16 * max(1, st.n), dtype=torch.uint8, device=st.pos.device)
                self.rec_alt = torch.empty_like(self.rec)
            # records known current: no conversion launch at all (verified on the device)
            drift = md.drift_params(self.pos_alt, st.pos_ref, self.dt, self.half_skin,
                                    self.walls, rec_in=self.rec if carry else None,
                                    rec_out=self.rec_alt if carry else None,
                                    rec_current=carry and self.rec_fresh,
                                    langevin=self.langevin)
            if self.pot is None:
                md.md_lj_forces(st, self.lj, self.nl, self.inv_mass, 0.5 * self.dt, kick=True,
                                ev=self.ev if ev else None, ev_cap=self.ev_cap, drift=drift)
            else:
                md.md_eam_forces(st, self.pot, self.nl, self.table, None, self.inv_mass,
                                 0.5 * self.dt, kick=True, ev=self.ev if ev else None,
                                 ev_cap=self.ev_cap, drift=drift)
            st.pos, self.pos_alt = self.pos_alt, st.pos
            if carry:
                self.rec, self.rec_alt = self.rec_alt, self.rec
                self.rec_fresh = True
            self.primed = True
        else:
            self.forces(kick=True, ev=ev)
        self.n_steps += 1
        if not self._capturing:
            self.eager_steps += 1

    def previous_positions(self):
        """Fused mode: positions at the last completed step (x(n)), by original id."""
        if not (self.fused and self.primed):
            return self.state.positions()
        return self.pos_alt[:, :3].cpu().numpy()[self.state._order()]

    # -- graphs ---------------------------------------------------------------
    def capture(self, steps, ev=True, tail=False):
        """Capture `steps` consecutive steps into one graph (for rebuild_every = k the graph
        must start at a multiple of k and span a multiple of k steps; in fused mode it must
        span an even number of steps, after at least one step, so that the two position
        buffers are back in place at the end of each replay).

        tail=True captures a graph that is replayed exactly once, as the last graph of a
        timed run (see prepare_timed): it may span any number of steps from an aligned
        start; it is returned and not kept as self.graph."""
        k = self.rebuild_every
        if k > 0 and ((steps % k and not tail) or self.n_steps % k):
            raise ValueError("graph of %d steps at step %d does not align with rebuilds every %d"
                             % (steps, self.n_steps, k))
        if self.fused and ((steps % 2 and not tail) or not self.primed):
            raise ValueError("fused mode: graphs span an even number of steps, after the first")
        n0 = self.n_steps
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        self._capturing = True
        try:
            with torch.cuda.graph(g, stream=s):
                for _ in range(steps):
                    self.step(ev)
        finally:
            self._capturing = False
        torch.cuda.current_stream().wait_stream(s)
        self.n_steps = n0  # capture recorded the steps; replays perform them
        if not tail:
            self.graph, self.graph_steps = g, steps
        return g

    def prepare_timed(self, n_steps, graph_steps, ev=True):
        """Graphs for a run of exactly n_steps steps made of replays only
        (timed_graph_plan): the main graph of G steps (captured now, and kept) and, when
        n_steps is not a multiple of G, a tail graph.  The run must start at a multiple of
        the graph period (after the first step in fused mode).  Returns the replay list
        [(graph, steps), ...]; run it with replay_timed() before any other step: capturing
        a tail of an odd number of fused steps leaves the position buffers as they will be
        after the whole run."""
        k = max(1, self.rebuild_every)
        if self.n_steps % k or (self.fused and not self.primed):
            raise ValueError("a timed run starts at a multiple of the rebuild period %d" % k)
        G, q, r = timed_graph_plan(n_steps, self.rebuild_every, self.fused, graph_steps)
        plan = []
        if q:
            if self.graph is None or self.graph_steps != G:
                self.capture(G, ev)
            plan += [(self.graph, G)] * q
        if r:
            plan.append((self.capture(r, ev, tail=True), r))
            if self.fused and r % 2:
                # the buffers end the run swapped: the main graph (held by the plan) must not
                # be replayed after it, so later runs capture afresh
                self.graph, self.graph_steps = None, 0
        return plan

    def align(self, ev=True):
        """Eager steps until the next step starts a rebuild period (and, in fused mode, the
        first step is done); returns how many were taken."""
        k = max(1, self.rebuild_every)
        taken = 0
        while (self.fused and not self.primed) or self.n_steps % k:
            self.step(ev)
            taken += 1
        return taken

    def replay_timed(self, plan, events=None):
        """Replay a prepare_timed() list; events (optional, len(plan) + 1 torch events) are
        recorded before the first and after every replay."""
        if events is not None:
            events[0].record()
        for q, (g, steps) in enumerate(plan):
            g.replay()
            self.n_steps += steps
            if events is not None:
                events[q + 1].record()

    def run(self, n_steps, graph_steps=0, ev=True):
        k = self.rebuild_every
        if self.fused and graph_steps:
            if not self.primed and n_steps > 0:
                self.step(ev)
                n_steps -= 1
            period = 2 * k // math.gcd(2, k) if k > 0 else 2
            graph_steps = max(period, graph_steps // period * period)
            while n_steps > 0 and k > 0 and self.n_steps % k:  # align to the rebuild period
                self.step(ev)
                n_steps -= 1
        elif k > 0 and graph_steps:
            graph_steps = max(k, graph_steps // k * k)
            while n_steps > 0 and self.n_steps % k:  # align to the rebuild period
                self.step(ev)
                n_steps -= 1
        if graph_steps and n_steps >= graph_steps:
            if self.graph is None or self.graph_steps != graph_steps:
                self.capture(graph_steps, ev)
            for _ in range(n_steps // graph_steps):
                self.graph.replay()
                self.n_steps += graph_steps
            rest = n_steps % graph_steps
        else:
            rest = n_steps
        for _ in range(rest):
            self.step(ev)

    # -- results --------------------------------------------------------------
    def energies(self, steps):
        """Per-step records {E_pot, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz, K} (eV) of the given
        step numbers (which must be within the last ev_cap)."""
        ev = md.ev_values(self.ev)[:, 0, :]
        rows = [ev[s % self.ev_cap] for s in steps]
        return np.array(rows)
