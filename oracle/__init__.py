"""FP64 CPU oracle of the photon-migration hot path (ctypes front end).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it.  The product library never imports, links or calls it, and it
never imports the product.  The arithmetic lives in ``oracle.c`` (plain C,
double precision, one photon at a time); this file only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB names another build of oracle.c; the mutation tests use it to run the
# pins against copies of the oracle with a planted mistake
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

# integer channels (units of 2^-31 launch weight unless a count)
ICH = ["R", "T", "A", "RR", "lost", "esc_w", "esc_w_gtL", "esc_n", "esc_n_gtL", "steps", "interactions",
       "gated"]
# floating channels
DCH = ["esc_w_void_path", "path_total", "path_solid", "path_void"]

EVENTS = {0: "face_x", 1: "face_y", 2: "face_z", 3: "scatter", 4: "esc_R", 5: "esc_T",
          6: "dead_absorb", 7: "dead_roulette", 8: "lost", 9: "gated",
          10: "reflect_x", 11: "reflect_y", 12: "reflect_z"}
#: boundary models: the plain one (periodic laterals, index 1, no pads, no gate) and the
#: paper's (air pads, Fresnel at index steps, mirror or periodic laterals, time gate)
BOUNDARY_PLAIN, BOUNDARY_PAPER = 0, 1
W1 = 2 ** 31


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("mask", ctypes.c_void_p),
                ("mu_s", ctypes.c_double), ("mu_a", ctypes.c_double), ("g", ctypes.c_double),
                ("w_roulette", ctypes.c_double), ("roulette_m", ctypes.c_uint32),
                ("path_cap", ctypes.c_double), ("source", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("max_steps", ctypes.c_uint32),
                ("boundary", ctypes.c_int32), ("lateral", ctypes.c_int32),
                ("n_solid", ctypes.c_double), ("gate", ctypes.c_double)]


REC_DTYPE = np.dtype([("ix", "<i4"), ("iy", "<i4"), ("iz", "<i4"), ("event", "<i4"),
                      ("fx", "<f8"), ("fy", "<f8"), ("fz", "<f8"),
                      ("ux", "<f8"), ("uy", "<f8"), ("uz", "<f8"),
                      ("d", "<f8"), ("tie_gap", "<f8"), ("w", "<i8"), ("k", "<u4"), ("pad", "<u4")])
PHOTON_DTYPE = np.dtype([("R", "<i8"), ("T", "<i8"), ("A", "<i8"), ("RR", "<i8"), ("lost", "<i8"),
                         ("w_final", "<i8"), ("steps", "<u8"), ("interactions", "<u8"),
                         ("path_void", "<f8"), ("path_solid", "<f8"), ("min_gap", "<f8"),
                         ("max_visit", "<f8"), ("fate", "<i4"), ("pad", "<i4")])


STATE_DTYPE = np.dtype([("ix", "<i8"), ("iy", "<i8"), ("iz", "<i8"),
                        ("fx", "<f8"), ("fy", "<f8"), ("fz", "<f8"), ("ux", "<f8"), ("uy", "<f8"), ("uz", "<f8"),
                        ("tau", "<f8"), ("w", "<i8"), ("k", "<u4"), ("pad", "<u4"), ("steps", "<u8"),
                        ("l_void", "<f8"), ("l_solid", "<f8"), ("score_s", "<f8"), ("score_a", "<f8"),
                        ("score_g", "<f8"), ("l_opt", "<f8"), ("nf", "<u4"), ("pad2", "<u4")])


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C11, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-pthread", _SRC, "-o", _LIB, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_void_p]
        L.orc_trace.restype = ctypes.c_int
        L.orc_trace.argtypes = [ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.c_void_p]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.POINTER(Problem), ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_fresnel.restype = ctypes.c_double
        L.orc_fresnel.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_double)]
        L.orc_philox.restype = None
        L.orc_philox.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        assert L.orc_sizeof_rec() == REC_DTYPE.itemsize
        assert L.orc_sizeof_photon() == PHOTON_DTYPE.itemsize
        assert L.orc_sizeof_problem() == ctypes.sizeof(Problem)
        assert L.orc_sizeof_state() == STATE_DTYPE.itemsize
        _lib = L
    return _lib


def philox(counter, key) -> np.ndarray:
    """Philox4x32-10 of one 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def fresnel(n1: float, n2: float, cos_i: float):
    """Unpolarised Fresnel reflectance from index n1 into n2 at incidence cosine cos_i,
    and the transmission cosine (0 under total internal reflection)."""
    ct = ctypes.c_double(0.0)
    r = lib().orc_fresnel(float(n1), float(n2), float(cos_i), ctypes.byref(ct))
    return r, ct.value


def _f32(x: float) -> float:
    """The transport sees its coefficients as float32; the oracle uses the same values."""
    return float(np.float32(x))


def make_problem(mask: np.ndarray, mu_s: float, mu_a: float, g: float, seed: int, stream_id: int = 0,
                 w_roulette: float = 1e-4, roulette_m: int = 10, path_cap: float = 0.0, source: int = 0,
                 max_steps: int = 1 << 24, boundary: int = BOUNDARY_PLAIN, lateral: int = 0,
                 n_solid: float = 1.0, gate: float = float("inf")):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    assert m.ndim == 3
    nz, ny, nx = m.shape
    P = Problem(nx=nx, ny=ny, nz=nz, mask=m.ctypes.data, mu_s=_f32(mu_s), mu_a=_f32(mu_a), g=_f32(g),
                w_roulette=_f32(w_roulette), roulette_m=roulette_m, path_cap=float(path_cap),
                source=source, seed=seed, stream_id=stream_id, max_steps=max_steps,
                boundary=boundary, lateral=lateral, n_solid=_f32(n_solid), gate=float(gate))
    return P, m


def run(mask, mu_s, mu_a, g, n_photons, seed, photon_begin=0, stream_id=0, nthreads=None, nbatch=1,
        fluence=True, grad=False, depth=False, **kw):
    """Run photons [photon_begin, photon_begin + n_photons) through the FP64 oracle.

    Returns a dict: per-batch integer channels ``ich`` [nbatch, len(ICH)], floating
    channels ``dch`` [nbatch, len(DCH)], and optionally ``fluence`` [nbatch, nz, ny, nx]
    (weight in units of 2^-31 times voxel), ``grad`` [nbatch, 3, 2, nz] and ``depth``
    [nbatch, 2, nz].  Photon p belongs to batch p mod nbatch.
    """
    P, m = make_problem(mask, mu_s, mu_a, g, seed, stream_id, **kw)
    nz, ny, nx = m.shape
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0)) or 1
    out = {}
    F = np.zeros((nbatch, nz, ny, nx), dtype=np.float64) if fluence else None
    G = np.zeros((nbatch, 3, 2, nz), dtype=np.float64) if grad else None
    D = np.zeros((nbatch, 2, nz), dtype=np.float64) if depth else None
    ich = np.zeros((nbatch, len(ICH)), dtype=np.int64)
    dch = np.zeros((nbatch, len(DCH)), dtype=np.float64)
    rc = lib().orc_run(ctypes.byref(P), photon_begin, n_photons, nthreads, nbatch,
                       F.ctypes.data if F is not None else None,
                       G.ctypes.data if G is not None else None,
                       D.ctypes.data if D is not None else None,
                       ich.ctypes.data, dch.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    out["ich"], out["dch"] = ich, dch
    if F is not None:
        out["fluence"] = F
    if G is not None:
        out["grad"] = G
    if D is not None:
        out["depth"] = D
    out["nthreads"] = nthreads
    return out


def totals(res) -> dict:
    """Sum the batch dimension of the channels into a name -> value dict."""
    d = {name: int(v) for name, v in zip(ICH, res["ich"].sum(axis=0))}
    d.update({name: float(v) for name, v in zip(DCH, res["dch"].sum(axis=0))})
    return d


def trace(mask, mu_s, mu_a, g, photon_ids, seed, max_rec=64, stream_id=0, **kw):
    """Per-step records (first ``max_rec`` steps) and per-photon summaries of the given photons."""
    P, m = make_problem(mask, mu_s, mu_a, g, seed, stream_id, **kw)
    ids = np.ascontiguousarray(np.asarray(photon_ids, dtype=np.uint64))
    n = ids.size
    recs = np.zeros((n, max_rec), dtype=REC_DTYPE)
    recs["event"] = -1
    summ = np.zeros(n, dtype=PHOTON_DTYPE)
    rc = lib().orc_trace(ctypes.byref(P), ids.ctypes.data, n, max_rec, recs.ctypes.data, summ.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return recs, summ


def step_from(mask, mu_s, mu_a, g, photon_id, state, seed, stream_id=0, **kw):
    """One oracle step of photon ``photon_id`` from ``state`` (a STATE_DTYPE record).

    Returns (event, new_state, tie_gap)."""
    P, m = make_problem(mask, mu_s, mu_a, g, seed, stream_id, **kw)
    st = np.array(state, dtype=STATE_DTYPE).reshape(1).copy()
    gap = ctypes.c_double(0.0)
    ev = lib().orc_step(ctypes.byref(P), int(photon_id), st.ctypes.data, ctypes.byref(gap))
    if ev < 0:
        raise ValueError("oracle rejected the problem")
    return ev, st[0], gap.value
