"""ctypes declarations of libmd950 (include/md.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmd950.so")

MD_OK = 0
MD_FP64, MD_FP32 = 0, 1
MD_ALWAYS, MD_IF_FLAGGED = 0, 1
MD_KICK_DRIFT, MD_KICK = 0, 1
MD_EV_LEN = 8
MD_EV_SCALE = 2.0 ** 36  # fixed-point units per eV of the per-box records
MD_TILE = 64
MD_NN_IMG = 1 << 30
FLAG_NEIGH_OVERFLOW, FLAG_TABLE_RANGE, FLAG_WALL, FLAG_NONFINITE, FLAG_STALE_LIST = 1, 2, 4, 8, 16
FLAG_STALE_RECORDS = 32
MD_ERR_ARG = -1
MD_DRIFT_MAX_BLOCKS = 32768
MD_ERR_STALE_LIST = -9
MD_ERR_STALE_RECORDS = -10
MD_ERR_WORKSPACE = -8
MD_NOALLOC_MAX_ATOMS = 1 << 20
MD_NOALLOC_MAX_TILES = 32768


class MDError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, _status_string(status), status))


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3), ("periodic", C.c_int * 3),
                ("pad", C.c_int)]


class Domain(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3), ("inv_len", C.c_double * 3),
                ("inv_w", C.c_double * 3), ("nc", C.c_int * 3), ("periodic", C.c_int * 3),
                ("cell_off", C.c_int), ("atom_off", C.c_int), ("n_atoms", C.c_int),
                ("tile_off", C.c_int), ("n_tiles", C.c_int), ("pad", C.c_int)]


class Tile(C.Structure):
    _fields_ = [("rep", C.c_int), ("first", C.c_int), ("count", C.c_int), ("pad", C.c_int)]


class Batch(C.Structure):
    _fields_ = [("n_rep", C.c_int), ("n_atoms", C.c_int), ("n_cells", C.c_int),
                ("n_tiles", C.c_int), ("tile_atoms", C.c_int), ("pad", C.c_int),
                ("r_ns", C.c_double), ("domains", C.c_void_p), ("tiles", C.c_void_p)]


class NList(C.Structure):
    _fields_ = [("neigh", C.c_void_p), ("nneigh", C.c_void_p), ("max_neigh", C.c_int),
                ("lanes", C.c_int), ("block", C.c_int)]


class Spline(C.Structure):
    _fields_ = [("coef", C.c_void_p), ("ncoef", C.c_int), ("pad", C.c_int), ("x_lo", C.c_double),
                ("h", C.c_double)]


class EAM(C.Structure):
    _fields_ = [("phi", Spline), ("rho", Spline), ("emb", Spline), ("r_cut", C.c_double)]


class LJ(C.Structure):
    _fields_ = [("eps", C.c_double), ("sigma", C.c_double), ("r_cut", C.c_double)]


class Walls(C.Structure):
    _fields_ = [("enabled", C.c_int), ("axis", C.c_int), ("piston_z0", C.c_double),
                ("piston_v", C.c_double), ("top", C.c_double)]


MD_MAX_THERMO_REGIONS = 4
MD_PROF_LEN = 18
PROF_FIELDS = ("N", "M", "ux", "uy", "uz", "Tx", "Ty", "Tz", "T", "Pxx", "Pyy", "Pzz", "Pxy",
               "Pxz", "Pyz", "P", "Epot_per_mass", "Eint_per_mass")


class ThermoRegion(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("temperature", C.c_double),
                ("gamma", C.c_double), ("u", C.c_double * 3)]


class Langevin(C.Structure):
    _fields_ = [("id", C.c_void_p), ("seed", C.c_ulonglong), ("axis", C.c_int),
                ("n_regions", C.c_int), ("region", ThermoRegion * MD_MAX_THERMO_REGIONS)]


MD_BPNN_MAX_G = 64


class BPNN(C.Structure):
    _fields_ = [("r_cut", C.c_double), ("r_s", C.c_double), ("n_g2", C.c_int), ("n_g4", C.c_int),
                ("h1", C.c_int), ("h2", C.c_int), ("g2_eta", C.c_double * MD_BPNN_MAX_G),
                ("g4_zeta", C.c_double * MD_BPNN_MAX_G), ("g4_lambda", C.c_double * MD_BPNN_MAX_G),
                ("g4_eta", C.c_double * MD_BPNN_MAX_G), ("weights", C.c_void_p)]


class Drift(C.Structure):
    _fields_ = [("pos_out", C.c_void_p), ("pos_ref", C.c_void_p), ("dt", C.c_double),
                ("half_skin", C.c_double), ("walls", Walls), ("rec_in", C.c_void_p),
                ("rec_out", C.c_void_p), ("rec_current", C.c_int), ("pad", C.c_int),
                ("langevin", C.c_void_p)]


_lib = None
_vp, _i, _d, _sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_P = C.POINTER

_SIGS = {
    "md_plan_count": (_i, [_i, _P(Box), _P(C.c_int), _d, _i, _P(C.c_int), _P(C.c_int)]),
    "md_plan": (_i, [_i, _P(Box), _P(C.c_int), _d, _i, _P(Domain), _P(Tile)]),
    "md_ctl_bytes": (_sz, []),
    "md_ctl_init": (_i, [_vp, _vp]),
    "md_workspace_bytes": (_sz, [_P(Batch)]),
    "md_eam_table_bytes": (_sz, [_P(EAM), _i]),
    "md_spline_fit": (_i, [_vp, _i, _d, _d, _d, _vp, _vp]),
    "md_eam_prepare": (_i, [_P(EAM), _i, _vp, _vp]),
    "md_bin_cells": (_i, [_P(Batch), _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_build_neighbors": (_i, [_P(Batch), _i, _vp, _vp, _P(NList), _vp, _vp]),
    "md_lj_forces": (_i, [_P(Batch), _P(LJ), _i, _vp, _P(NList), _vp, _vp, _d, _d, _P(Drift),
                          _vp, _i, _vp, _vp, _vp]),
    "md_eam_forces": (_i, [_P(Batch), _P(EAM), _i, _vp, _vp, _P(NList), _vp, _vp, _vp, _d, _d,
                           _P(Drift), _vp, _i, _vp, _vp, _vp]),
    "md_eam_forces_noalloc": (_i, [_P(Batch), _P(EAM), _i, _vp, _vp, _P(NList), _vp, _vp, _vp,
                                   _d, _d, _P(Drift), _vp, _i, _vp, _vp]),
    "md_verlet_step": (_i, [_P(Batch), _i, _d, _vp, _vp, _vp, _i, _d, _P(Walls), _P(Langevin),
                            _vp, _d, _vp, _vp]),
    "md_eam_backward": (_i, [_P(Batch), _P(EAM), _i, _vp, _P(NList), _vp, _vp, _vp, _vp, _vp,
                             _vp]),
    "md_backward_workspace_bytes": (_sz, [_P(Batch), _P(EAM)]),
    "md_eam_backward_jac": (_i, [_P(Batch), _P(EAM), _i, _vp, _P(NList), _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp]),
    "md_density_jacobian_bytes": (_sz, [_P(Batch), _P(EAM)]),
    "md_eam_density_jacobian": (_i, [_P(Batch), _P(EAM), _vp, _P(NList), _vp, _vp, _vp]),
    "md_eam_forces_jac": (_i, [_P(Batch), _P(EAM), _i, _vp, _vp, _P(NList), _vp, _vp, _vp, _vp,
                               _vp, _vp]),
    "md_force_loss_workspace_bytes": (_sz, [_i]),
    "md_force_loss": (_i, [_i, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
    "md_atom_observables": (_i, [_P(Batch), _P(EAM), _P(LJ), _vp, _P(NList), _vp, _vp, _vp,
                                 _vp, _vp]),
    "md_profile_workspace_bytes": (_sz, [_i]),
    "md_bpnn_workspace_bytes": (_sz, [_P(Batch), _P(BPNN)]),
    "md_bpnn_forces": (_i, [_P(Batch), _P(BPNN), _vp, _P(NList), _vp, _vp, _vp, _d, _d, _vp, _i,
                            _vp, _vp, _vp]),
    "md_profiles": (_i, [_P(Batch), _i, _d, _d, _i, _vp, _vp, _d, _vp, _vp, _vp, _vp, _vp]),
    "md_read_flags": (_i, [_vp, _P(C.c_int), _vp]),
    "md_clear_flags": (_i, [_vp, _vp]),
    "md_status_string": (C.c_char_p, [_i]),
    "md_timer_arm": (_i, [_i]),
    "md_timer_read": (_i, [_P(C.c_float)]),
}

MD_KERNEL = {"bin_count": 1, "build": 2, "lj": 3, "eam_density": 4, "eam_force": 5,
             "kick_drift": 6, "eam_adjoint": 7, "bpnn_desc": 8, "bpnn_force": 9}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmd950.so is not built (run paper_2511_22951_amd/build.py); "
                               "the MD path has no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _status_string(s):
    try:
        return lib().md_status_string(int(s)).decode()
    except Exception:  # pragma: no cover
        return "status"


def check(status, what=""):
    if status != MD_OK:
        raise MDError(status, what)
    return status
