"""The C-ABI library loads and exports every symbol include/md.h declares; host-only
entry points (planning, sizes, status strings) work without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2511_22951_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("libmd950.so not built; run __graft_entry__.build()")
    return _native.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for nm in names:
        assert hasattr(lib, nm), nm
    from paper_2511_22951_amd import _native
    assert set(names) == set(_native.EXPORTED)


def test_plan_on_host(lib):
    from paper_2511_22951_amd import _native as N
    import mdinputs as mi
    pos, box = mi.fcc_lattice(32, 32, 32, 3.615)
    b = (N.Box * 1)()
    for a in range(3):
        b[0].lo[a], b[0].len[a], b[0].periodic[a] = 0.0, box.len[a], 1
    off = (C.c_int * 2)(0, len(pos))
    nc, nt = C.c_int(), C.c_int()
    assert lib.md_plan_count(1, b, off, 5.8, 64, C.byref(nc), C.byref(nt)) == 0
    assert nc.value == 19 ** 3 and nt.value == len(pos) // 64
    doms = (N.Domain * 1)()
    tiles = (N.Tile * nt.value)()
    assert lib.md_plan(1, b, off, 5.8, 64, doms, tiles) == 0
    assert tuple(doms[0].nc) == (19, 19, 19)
    assert tiles[nt.value - 1].first == len(pos) - 64 and tiles[5].count == 64


def test_plan_rejects_small_box_and_bad_args(lib):
    from paper_2511_22951_amd import _native as N
    b = (N.Box * 1)()
    for a in range(3):
        b[0].len[a], b[0].periodic[a] = 11.0, 1
    off = (C.c_int * 2)(0, 100)
    nc, nt = C.c_int(), C.c_int()
    assert lib.md_plan_count(1, b, off, 5.8, 64, C.byref(nc), C.byref(nt)) == -2  # MD_ERR_BOX
    assert lib.md_plan_count(1, b, off, 5.0, 32, C.byref(nc), C.byref(nt)) == -1  # tile size
    b[0].periodic[0] = 0  # a non-periodic axis does not need L > 2 r_ns
    b[0].periodic[1] = 0
    b[0].periodic[2] = 0
    assert lib.md_plan_count(1, b, off, 5.8, 64, C.byref(nc), C.byref(nt)) == 0
    assert lib.md_status_string(-3).decode().startswith("neighbour list overflow")


def test_batch_plan_tiles_never_straddle_boxes(lib):
    from paper_2511_22951_amd import _native as N
    import mdinputs as mi
    reps = mi.cold_curve_replicas()
    n = len(reps)
    b = (N.Box * n)()
    offs = [0]
    for r, rep in enumerate(reps):
        for a in range(3):
            b[r].len[a], b[r].periodic[a] = rep.box.len[a], 1
        offs.append(offs[-1] + len(rep.pos))
    off = (C.c_int * (n + 1))(*offs)
    nc, nt = C.c_int(), C.c_int()
    assert lib.md_plan_count(n, b, off, 5.8, 64, C.byref(nc), C.byref(nt)) == 0
    doms = (N.Domain * n)()
    tiles = (N.Tile * nt.value)()
    assert lib.md_plan(n, b, off, 5.8, 64, doms, tiles) == 0
    for t in range(nt.value):
        T = tiles[t]
        d = doms[T.rep]
        assert d.atom_off <= T.first and T.first + T.count <= d.atom_off + d.n_atoms
    assert sum(doms[r].n_tiles for r in range(n)) == nt.value


def test_noalloc_entry_point_rejects_oversize_batches(lib):
    """md_eam_forces_noalloc refuses batches beyond its static scratch with MD_ERR_WORKSPACE,
    on the host, before any device work."""
    from paper_2511_22951_amd import _native as N
    dummy = C.c_void_p(0x1000)
    for n_atoms, n_tiles in ((N.MD_NOALLOC_MAX_ATOMS + 1, 16385), (1000, N.MD_NOALLOC_MAX_TILES + 1)):
        b = N.Batch(1, n_atoms, 8, n_tiles, 64, 0, 5.8, dummy, dummy)
        st = lib.md_eam_forces_noalloc(C.byref(b), None, 1, None, None, None, None, None, None,
                                       0.0, 0.0, None, None, 1, None, None)
        assert st == N.MD_ERR_WORKSPACE


def test_force_matching_entry_points_check_arguments_on_the_host(lib):
    """The force-matching entry points reject malformed arguments with MD_ERR_ARG (or a zero
    size) before any device work: a NULL Jacobian, more than 128 rho coefficients for the
    Jacobian forms, a negative atom count or NULL outputs for the loss."""
    from paper_2511_22951_amd import _native as N
    dummy = C.c_void_p(0x1000)
    b = N.Batch(1, 1000, 8, 16, 64, 0, 5.8, dummy, dummy)
    sp = N.Spline(dummy, 64, 0, 1.5, 4.0 / 61)
    big = N.Spline(dummy, 200, 0, 1.5, 4.0 / 197)
    p = N.EAM(sp, sp, N.Spline(dummy, 64, 0, 5.0, 20.0 / 61), 5.5)
    p_big = N.EAM(big, big, N.Spline(dummy, 64, 0, 5.0, 20.0 / 61), 5.5)
    assert lib.md_density_jacobian_bytes(C.byref(b), C.byref(p)) == (8 * 1000 * 64 + 255) // 256 * 256
    assert lib.md_density_jacobian_bytes(C.byref(b), C.byref(p_big)) == 0
    nl = N.NList(dummy, dummy, 128, 4)
    assert lib.md_eam_density_jacobian(C.byref(b), C.byref(p_big), dummy, C.byref(nl), dummy,
                                       dummy, None) == N.MD_ERR_ARG
    assert lib.md_eam_forces_jac(C.byref(b), C.byref(p), 0, dummy, dummy, C.byref(nl), None,
                                 dummy, None, dummy, dummy, None) == N.MD_ERR_ARG
    assert lib.md_eam_forces_jac(C.byref(b), C.byref(p_big), 0, dummy, dummy, C.byref(nl), dummy,
                                 dummy, None, dummy, dummy, None) == N.MD_ERR_ARG
    assert lib.md_eam_backward_jac(C.byref(b), C.byref(p), 0, dummy, C.byref(nl), dummy, None,
                                   dummy, dummy, dummy, dummy, None) == N.MD_ERR_ARG
    assert lib.md_force_loss_workspace_bytes(-1) == 0
    assert lib.md_force_loss_workspace_bytes(300000) == 1024 * 8
    assert lib.md_force_loss(-1, 0, dummy, dummy, dummy, None, dummy, None) == N.MD_ERR_ARG
    assert lib.md_force_loss(10, 0, dummy, dummy, None, None, dummy, None) == N.MD_ERR_ARG
    assert lib.md_force_loss(10, 0, None, dummy, dummy, None, dummy, None) == N.MD_ERR_ARG
    assert lib.md_force_loss(10, 7, dummy, dummy, dummy, None, dummy, None) == N.MD_ERR_ARG
