"""Helpers for the GPU parity tests (they compare the HIP path, called through the
C ABI, with the oracle on the same seeded inputs)."""
import numpy as np

import mdinputs as mi
from oracle import core


def displaced(cells, a, sigma, seed, box_periodic=(1, 1, 1), shape=None):
    n1, n2, n3 = (cells, cells, cells) if shape is None else shape
    pos, box = mi.fcc_lattice(n1, n2, n3, a)
    box = mi.Box(box.lo, box.len, box_periodic)
    rng = np.random.default_rng(seed)
    x = pos + rng.normal(0, sigma, pos.shape)
    return mi.wrap_into_box(x, box), box


def neighbor_sets_by_id(state, nl):
    """{original id: sorted array of original ids} from the device list."""
    ids = state.id.cpu().numpy()
    lists = nl.host_lists()
    return {int(ids[i]): np.sort(ids[lists[i]]) for i in range(len(lists))}


def assert_same_sets(gpu_sets, oracle_lists):
    for i, want in enumerate(oracle_lists):
        got = gpu_sets[i]
        assert np.array_equal(got, want), (i, got, want)


def rel_fro(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def oracle_eam(pos, box, table):
    return core.eam(pos, box, core.EAMPotential.from_table(table))


def md_ev(n_rep=1, cap=1):
    """A per-step record buffer for cap steps of n_rep boxes (int64 fixed point)."""
    from paper_2511_22951_amd import md
    return md.ev_buffer(cap, n_rep)


def evv(ev):
    """Records in eV as float64 numpy."""
    from paper_2511_22951_amd import md
    return md.ev_values(ev)
