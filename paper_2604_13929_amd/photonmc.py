"""Python binding of libphotonmc.so (argument marshalling only).

Torch provides device memory and the current HIP stream; every step of the
walk and of the reduction runs in the library's HIP kernels.  If the library
is missing the calls raise: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from dataclasses import dataclass, field

import numpy as np
import torch

from . import build as _build

LIB_PATH = _build.LIB

MC_ACCUMULATE = 1
MC_TIMED = 2
MC_FP64 = 4
MC_DIRECT_DEPOSIT = 8
MC_LINE_STAGING = 16
#: Q31 units per deposit quantum: each segment's deposit is rounded to a multiple of it
ABI_VERSION = 4
DEPOSIT_QUANTUM = 256
GRAD_FIXED_BITS = 20        # score bins in units of 2^-20 Q31 weight x voxel
NSCALARS = 16
NSUMMARY = 32
SCALARS = ["R", "T", "A", "RR", "lost", "esc_w", "esc_w_gtL", "esc_w_void_path_lo", "esc_n", "esc_n_gtL",
           "steps", "interactions", "launched", "esc_w_void_path_hi", "gated"]
SUMMARY = ["phi3d", "phi1d", "phi_pore", "r", "porosity", "ratio", "identity_rhs", "R", "T", "A", "RR", "lost",
           "closure_exact", "front_back", "L_opt", "esc_frac", "Pw_void_gtL", "Pn_void_gtL", "mean_void_path",
           "steps_per_photon", "interactions_per_photon", "status", "n_solid", "launched", "gated"]
BOUNDARY_PLAIN, BOUNDARY_PAPER = 0, 1
LATERAL_PERIODIC, LATERAL_MIRROR = 0, 1
#: trace events
EVENTS = {0: "face_x", 1: "face_y", 2: "face_z", 3: "scatter", 4: "esc_R", 5: "esc_T", 6: "dead_absorb",
          7: "dead_roulette", 8: "lost", 9: "gated", 10: "reflect_x", 11: "reflect_y", 12: "reflect_z"}
SPEED_OF_LIGHT = 299_792_458.0
W1 = 2 ** 31


class McVolume(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("mask", ctypes.c_void_p)]


class McOptics(ctypes.Structure):
    _fields_ = [("mu_s", ctypes.c_float), ("mu_a", ctypes.c_float), ("g", ctypes.c_float),
                ("w_roulette", ctypes.c_float), ("roulette_m", ctypes.c_uint32), ("path_cap", ctypes.c_float),
                ("source", ctypes.c_int32), ("max_steps", ctypes.c_uint32),
                ("boundary", ctypes.c_int32), ("lateral", ctypes.c_int32), ("n_solid", ctypes.c_float),
                ("reserved", ctypes.c_int32), ("gate", ctypes.c_double)]


class McChGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("dt", ctypes.c_double)]


class McTune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("defer", ctypes.c_int32)]


class McJob(ctypes.Structure):
    _fields_ = [("vol", McVolume), ("opt", McOptics), ("photon_begin", ctypes.c_uint64),
                ("n_photons", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("accumulate", ctypes.c_int32), ("fluence", ctypes.c_void_p), ("scalars", ctypes.c_void_p),
                ("summary", ctypes.c_void_p), ("depth", ctypes.c_void_p)]


class McEscapeBins(ctypes.Structure):
    _fields_ = [("bin_width", ctypes.c_double), ("nbins", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("hist_w", ctypes.c_void_p), ("hist_n", ctypes.c_void_p)]


MAX_BATCH_JOBS = 64

TRACE_DTYPE = np.dtype([("fx", "<f8"), ("fy", "<f8"), ("fz", "<f8"), ("ux", "<f8"), ("uy", "<f8"), ("uz", "<f8"),
                        ("d", "<f8"), ("s_rem", "<f8"), ("w", "<u4"), ("k", "<u4"),
                        ("ix", "<i4"), ("iy", "<i4"), ("iz", "<i4"), ("event", "<i4")])
PHOTON_DTYPE = np.dtype([("R", "<i8"), ("T", "<i8"), ("A", "<i8"), ("RR", "<i8"), ("lost", "<i8"),
                         ("w_final", "<u4"), ("fate", "<u4"), ("steps", "<u4"), ("interactions", "<u4"),
                         ("path_void", "<f8"), ("path_solid", "<f8")])

# exported symbols and their signatures (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "mc_abi_version": (ctypes.c_int, []),
    "mc_sizeof": (ctypes.c_size_t, [ctypes.c_char_p]),
    "mc_last_error": (ctypes.c_char_p, []),
    "mc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mc_tune_default": (None, [_P]),
    "mc_run_workspace_bytes": (ctypes.c_size_t, [_P]),
    "mc_run": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_int, _P, _P, _P, ctypes.c_size_t, _P, _P]),
    "mc_run_escape_histogram": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                               ctypes.c_uint32, ctypes.c_int, _P, _P, _P, ctypes.c_size_t, _P,
                                               ctypes.c_double, ctypes.c_int32, _P, _P, _P]),
    "mc_run_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_int, _P, _P, _P, _P]),
    "mc_run_noalloc_max_bricks": (ctypes.c_size_t, []),
    "mc_walk_elapsed_ms": (ctypes.c_int, [_P]),
    "mc_reduce_workspace_bytes": (ctypes.c_size_t, [_P]),
    "mc_reduce": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mc_probe_scatter": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _P]),
    "mc_probe_math": (ctypes.c_int, [_P, _P]),
    "mc_grad_workspace_bytes": (ctypes.c_size_t, [_P]),
    "mc_grad": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P]),
    "mc_batch_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "mc_run_batch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, _P, _P, ctypes.c_size_t, _P]),
    "mc_run_batch_escape_histogram": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, _P, _P, _P,
                                                     ctypes.c_size_t, _P]),
    "mc_autotune_batch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, _P, ctypes.c_size_t, _P, _P]),
    "mc_batch_graph_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, _P, _P, ctypes.c_size_t, _P]),
    "mc_graph_launch": (ctypes.c_int, [_P, _P]),
    "mc_graph_destroy": (ctypes.c_int, [_P]),
    "mc_trace": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                ctypes.c_int, _P, _P, _P, ctypes.c_size_t, _P]),
    # spinodal.h: the Cahn-Hilliard mask generator
    "mc_ch_workspace_bytes": (ctypes.c_size_t, [_P]),
    "mc_ch_init": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mc_ch_steps": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_size_t, ctypes.c_int, _P]),
    "mc_ch_field": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mc_ch_psd": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mc_ch_elapsed_ms": (ctypes.c_double, []),
    "mc_rank_threshold_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "mc_rank_threshold": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, _P, _P, ctypes.c_size_t, _P]),
    "mc_ch_generate_workspace_bytes": (ctypes.c_size_t, [_P]),
    # analytics.h: morphology and fluence analytics
    "mc_chord_histogram": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
    "mc_phase_contrast": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "mc_escape_path_histogram": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, _P,
                                                ctypes.c_int32, _P, _P, _P, _P, _P]),
    "mc_bright_colocalization": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P, _P]),
    "mc_pore_distance_workspace_bytes": (ctypes.c_size_t, [_P]),
    "mc_pore_distance": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, _P]),
    "mc_pore_spearman_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "mc_mask_psd_workspace_bytes": (ctypes.c_size_t, [_P]),
    "mc_mask_psd": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t, _P]),
    "mc_pore_spearman": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P]),
    "mc_ch_generate": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mc_ch_grid_from_target": (ctypes.c_int, [ctypes.c_double, _P]),
    "mc_psd_peak": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    # the paper's reference model and comparison metrics
    "mc_time_gate": (ctypes.c_int, [ctypes.c_double] * 7 + [_P]),
    "mc_da_profile": (ctypes.c_int, [ctypes.c_double] * 4 + [ctypes.c_int32, _P, _P]),
    "mc_rms_w": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
}

_lib = None


MC_OK, MC_WARN_LOST, MC_EINVAL, MC_EOVERFLOW, MC_EHIP, MC_ENOSPACE = 0, 1, -1, -2, -3, -4


class McError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class McLostWeightWarning(UserWarning):
    """Some weight was stopped by the step or path cap (summary status MC_WARN_LOST)."""


def _summary_status(status: float, where: str):
    """Act on summary[MC_Q_STATUS] as the reduction wrote it."""
    st = int(status)
    if st < 0:
        raise McError(st, where, load().mc_strerror(st).decode())
    if st == MC_WARN_LOST:
        warnings.warn(f"{where}: {load().mc_strerror(st).decode()}", McLostWeightWarning, stacklevel=3)


def load(path: str = LIB_PATH):
    """Load the HIP library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2604_13929_amd.build.build_library() "
                           "(or __graft_entry__.build()) first -- there is no fallback path")
    L = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.mc_abi_version() != ABI_VERSION:
        raise RuntimeError(f"ABI mismatch: {path} is version {L.mc_abi_version()}, the binding {ABI_VERSION}; "
                           "rebuild the library")
    for name, size in (("mc_volume", ctypes.sizeof(McVolume)), ("mc_optics", ctypes.sizeof(McOptics)),
                       ("mc_job", ctypes.sizeof(McJob)), ("mc_escape_bins", ctypes.sizeof(McEscapeBins)),
                       ("mc_tune", ctypes.sizeof(McTune)), ("mc_trace_rec", TRACE_DTYPE.itemsize),
                       ("mc_photon_rec", PHOTON_DTYPE.itemsize), ("mc_ch_grid", ctypes.sizeof(McChGrid))):
        if L.mc_sizeof(name.encode()) != size:
            raise RuntimeError(f"ABI mismatch: sizeof({name}) is {L.mc_sizeof(name.encode())}, binding has {size}")
    _lib = L
    return L


def exported_symbols():
    return list(_SIGS)


def _check(status: int, where: str):
    if status < 0:
        L = load()
        raise McError(status, where, (L.mc_last_error() or b"").decode() or L.mc_strerror(status).decode())
    return status


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Optics:
    """Solid-phase optics per voxel length; pores are transparent.  ``boundary``
    selects the plain model (periodic laterals, index 1) or the paper's (air pads,
    ``lateral`` mirrors or periodic faces, solid index ``n_solid`` with Fresnel
    reflection and refraction, optional time gate ``gate`` = c t_end in voxels)."""
    mu_s: float
    mu_a: float
    g: float
    w_roulette: float = 1e-4
    roulette_m: int = 10
    path_cap: float = 0.0
    source: int = 0
    max_steps: int = 0
    boundary: int = BOUNDARY_PLAIN
    lateral: int = LATERAL_PERIODIC
    n_solid: float = 0.0
    gate: float = 0.0

    def c(self) -> McOptics:
        return McOptics(self.mu_s, self.mu_a, self.g, self.w_roulette, self.roulette_m, self.path_cap,
                        self.source, self.max_steps, self.boundary, self.lateral, self.n_solid, 0, self.gate)


def paper_optics(mu_s: float, mu_a: float, g: float, n_solid: float = 1.746, lateral: int = LATERAL_MIRROR,
                 gate: float = 0.0, **kw) -> Optics:
    """Optics under the paper's boundary model (mirrors, air pads, Fresnel at the solid's
    index, gate in voxels of optical path or 0 for none)."""
    return Optics(mu_s, mu_a, g, boundary=BOUNDARY_PAPER, lateral=lateral, n_solid=n_solid, gate=gate, **kw)


def time_gate_seconds(mu_a: float, mu_s_red: float, porosity: float, thickness: float, n_eff: float,
                      c: float = SPEED_OF_LIGHT) -> float:
    """mc_time_gate (Eq. tend) for solid (shell) coefficients mu_a and mu_s' in SI
    units (1/m, m, s): t_end in seconds."""
    out = ctypes.c_double(0.0)
    _check(load().mc_time_gate(float(mu_s_red), float(mu_a), 0.0, float(porosity), float(thickness), float(n_eff),
                               float(c), ctypes.byref(out)), "mc_time_gate")
    return out.value


def time_gate_voxels(mu_s: float, mu_a: float, g: float, porosity: float, nz: int, n_eff: float) -> float:
    """mc_time_gate with c = 1 for solid coefficients per voxel and a slab of nz voxels:
    the optical path limit c t_end in voxels (what Optics.gate takes)."""
    out = ctypes.c_double(0.0)
    _check(load().mc_time_gate(float(mu_s), float(mu_a), float(g), float(porosity), float(nz), float(n_eff), 1.0,
                               ctypes.byref(out)), "mc_time_gate")
    return out.value


def da_profile(mu_s: float, mu_a: float, g: float, porosity: float, nz: int):
    """mc_da_profile (Sec. 2.4): the collimated-source diffusion approximation's
    Phi/S0 averaged over each of nz voxel layers, and L_opt in voxels."""
    prof = np.empty(int(nz), dtype=np.float64)
    l_opt = ctypes.c_double(0.0)
    _check(load().mc_da_profile(float(mu_s), float(mu_a), float(g), float(porosity), int(nz),
                                prof.ctypes.data_as(ctypes.c_void_p), ctypes.byref(l_opt)), "mc_da_profile")
    return prof, l_opt.value


@dataclass
class Tune:
    block: int = 0
    waves_per_cu: int = 0
    chunk: int = 0
    refill: int = 0
    defer: int = 0

    def c(self) -> McTune:
        return McTune(self.block, self.waves_per_cu, self.chunk, self.refill, self.defer)


@dataclass
class RunResult:
    """Device tallies of a run: fluence int64[nz][ny][nx] and int64[NSCALARS]."""
    fluence: torch.Tensor
    scalars: torch.Tensor
    walk_ms: float | None = None
    escape_hist_w: torch.Tensor | None = None   # int64[nbins] with escape_bins
    escape_hist_n: torch.Tensor | None = None

    def scalar_dict(self) -> dict:
        s = self.scalars.cpu().tolist()
        d = {name: int(s[i]) for i, name in enumerate(SCALARS)}
        d["esc_w_void_path"] = (d["esc_w_void_path_hi"] << 32) + (d["esc_w_void_path_lo"] % (1 << 64))
        return d


def volume(mask: torch.Tensor) -> McVolume:
    if mask.dtype != torch.uint8 or mask.dim() != 3 or not mask.is_cuda or not mask.is_contiguous():
        raise ValueError("mask must be a contiguous uint8 device tensor [nz, ny, nx]")
    nz, ny, nx = mask.shape
    return McVolume(nx, ny, nz, 0, mask.data_ptr())


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def run(mask: torch.Tensor, optics: Optics, n_photons: int, seed: int, photon_begin: int = 0, stream_id: int = 0,
        accumulate: RunResult | None = None, tune: Tune | None = None, timed: bool = False,
        fp64: bool = False, direct: bool = False, escape_bins: tuple[float, int] | None = None,
        line_staging: bool = False) -> RunResult:
    """mc_run on the current stream of the mask's device (fp64: the FP64 reference transport;
    direct: MC_DIRECT_DEPOSIT; line_staging: MC_LINE_STAGING).
    escape_bins = (bin_width, nbins): mc_run_escape_histogram, which also bins the
    in-pore path of the escaping photons into res.escape_hist_w / escape_hist_n."""
    L = load()
    vol = volume(mask)
    dev = mask.device
    if accumulate is None:
        res = RunResult(torch.empty(tuple(mask.shape), dtype=torch.int64, device=dev),
                        torch.empty(NSCALARS, dtype=torch.int64, device=dev))
        flags = 0
    else:
        res, flags = accumulate, MC_ACCUMULATE
    if timed:
        flags |= MC_TIMED
    if fp64:
        flags |= MC_FP64
    if direct:
        flags |= MC_DIRECT_DEPOSIT
    if line_staging:
        flags |= MC_LINE_STAGING
    nbytes = L.mc_run_workspace_bytes(ctypes.byref(vol))
    ws = workspace(nbytes, dev)
    opt = optics.c()
    t = tune.c() if tune is not None else None
    tref = ctypes.byref(t) if t is not None else None
    if escape_bins is None:
        _check(L.mc_run(ctypes.byref(vol), ctypes.byref(opt), photon_begin, n_photons, seed, stream_id, flags,
                        res.fluence.data_ptr(), res.scalars.data_ptr(), ws.data_ptr(), ws.numel(), tref,
                        _stream(dev)), "mc_run")
    else:
        width, nbins = float(escape_bins[0]), int(escape_bins[1])
        if res.escape_hist_w is None or res.escape_hist_w.numel() != nbins:
            if accumulate is not None:
                raise ValueError("accumulate needs a result that carries histograms of the same nbins")
            res.escape_hist_w = torch.empty(nbins, dtype=torch.int64, device=dev)
            res.escape_hist_n = torch.empty(nbins, dtype=torch.int64, device=dev)
        _check(L.mc_run_escape_histogram(ctypes.byref(vol), ctypes.byref(opt), photon_begin, n_photons, seed,
                                         stream_id, flags, res.fluence.data_ptr(), res.scalars.data_ptr(),
                                         ws.data_ptr(), ws.numel(), tref, width, nbins,
                                         res.escape_hist_w.data_ptr(), res.escape_hist_n.data_ptr(), _stream(dev)),
               "mc_run_escape_histogram")
    res._ws = ws  # keep the workspace alive with the queued work
    if timed:
        ms = ctypes.c_float(0.0)
        _check(L.mc_walk_elapsed_ms(ctypes.byref(ms)), "mc_walk_elapsed_ms")
        res.walk_ms = float(ms.value)
    return res


def run_noalloc(mask: torch.Tensor, optics: Optics, n_photons: int, seed: int, photon_begin: int = 0,
                stream_id: int = 0, accumulate: RunResult | None = None, tune: Tune | None = None,
                fp64: bool = False) -> RunResult:
    """mc_run_noalloc on the current stream: mc_run's tallies with no workspace (the
    library's fixed per-GPU scratch; calls on one GPU must not overlap)."""
    L = load()
    vol = volume(mask)
    dev = mask.device
    if accumulate is None:
        res = RunResult(torch.empty(tuple(mask.shape), dtype=torch.int64, device=dev),
                        torch.empty(NSCALARS, dtype=torch.int64, device=dev))
        flags = 0
    else:
        res, flags = accumulate, MC_ACCUMULATE
    if fp64:
        flags |= MC_FP64
    opt = optics.c()
    t = tune.c() if tune is not None else None
    _check(L.mc_run_noalloc(ctypes.byref(vol), ctypes.byref(opt), photon_begin, n_photons, seed, stream_id, flags,
                            res.fluence.data_ptr(), res.scalars.data_ptr(), ctypes.byref(t) if t is not None else None,
                            _stream(dev)), "mc_run_noalloc")
    return res


@dataclass
class Summary:
    values: dict
    depth: np.ndarray = field(repr=False)        # Phi/S0 per depth
    depth_solid: np.ndarray = field(repr=False)
    depth_pore: np.ndarray = field(repr=False)

    def __getitem__(self, k):
        return self.values[k]


def reduce_async(mask: torch.Tensor, res: RunResult):
    """mc_reduce into device buffers (summary double[NSUMMARY], depth double[3][nz])."""
    L = load()
    vol = volume(mask)
    dev = mask.device
    summary = torch.empty(NSUMMARY, dtype=torch.float64, device=dev)
    depth = torch.empty((3, mask.shape[0]), dtype=torch.float64, device=dev)
    ws = workspace(L.mc_reduce_workspace_bytes(ctypes.byref(vol)), dev)
    _check(L.mc_reduce(ctypes.byref(vol), res.fluence.data_ptr(), res.scalars.data_ptr(), summary.data_ptr(),
                       depth.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)), "mc_reduce")
    return summary, depth, ws


def reduce(mask: torch.Tensor, res: RunResult) -> Summary:
    summary, depth, ws = reduce_async(mask, res)
    s = summary.cpu().numpy()
    d = depth.cpu().numpy()
    del ws
    vals = {name: float(s[i]) for i, name in enumerate(SUMMARY)}
    _summary_status(vals["status"], "mc_reduce")
    return Summary(vals, d[0], d[1], d[2])


def trace(mask: torch.Tensor, optics: Optics, photon_ids, max_steps: int, seed: int, stream_id: int = 0,
          fp64: bool = False):
    """Per-step records [n, max_steps] and per-photon outcomes [n] (numpy structured arrays)."""
    L = load()
    vol = volume(mask)
    dev = mask.device
    ids = torch.as_tensor(np.asarray(photon_ids, dtype=np.uint64).view(np.int64), device=dev)
    n = int(ids.numel())
    recs = torch.empty((n, max_steps, TRACE_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    outc = torch.empty((n, PHOTON_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    ws = workspace(L.mc_run_workspace_bytes(ctypes.byref(vol)), dev)
    opt = optics.c()
    _check(L.mc_trace(ctypes.byref(vol), ctypes.byref(opt), ids.data_ptr(), n, max_steps, seed, stream_id,
                      MC_FP64 if fp64 else 0, recs.data_ptr(), outc.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)), "mc_trace")
    r = recs.cpu().numpy().reshape(-1).view(TRACE_DTYPE).reshape(n, max_steps)
    o = outc.cpu().numpy().reshape(-1).view(PHOTON_DTYPE)
    return r, o


def probe_scatter(table: torch.Tensor, n_ops: int, mode: int = 0, waves_per_cu: int = 16) -> float:
    """Time mc_probe_scatter on the current stream (HIP events on that stream);
    returns operations per second."""
    L = load()
    dev = table.device
    stream = torch.cuda.current_stream(dev)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    _check(L.mc_probe_scatter(table.data_ptr(), table.numel(), n_ops, mode, waves_per_cu, _stream(dev)),
           "mc_probe_scatter")
    stop.record(stream)
    stop.synchronize()
    threads = torch.cuda.get_device_properties(dev).multi_processor_count * waves_per_cu * 64
    done = max(1, n_ops // threads) * threads
    return done / (start.elapsed_time(stop) * 1e-3)


def probe_math(device: str | torch.device = "cuda:0") -> dict:
    """mc_probe_math: the largest errors of the FP32 transport's hardware sine,
    cosine (absolute), logarithm and square root (relative) over all 2^24 uniforms,
    against FP64."""
    L = load()
    out = torch.empty(4, dtype=torch.float64, device=device)
    _check(L.mc_probe_math(out.data_ptr(), _stream(out.device)), "mc_probe_math")
    return dict(zip(("sin", "cos", "log", "sqrt"), out.cpu().tolist()))


@dataclass
class BatchJob:
    """One job of a batch: a mask on the device, its optics, photons and stream."""
    mask: torch.Tensor
    optics: Optics
    n_photons: int
    seed: int
    stream_id: int = 0
    photon_begin: int = 0
    reduce: bool = True


class Batch:
    """Device buffers and the C job table of a batch (they must outlive queued work)."""

    def __init__(self, jobs: list[BatchJob], accumulate_into: "Batch | None" = None):
        if not 1 <= len(jobs) <= MAX_BATCH_JOBS:
            raise ValueError(f"a batch holds 1 to {MAX_BATCH_JOBS} jobs")
        self.jobs = jobs
        dev = jobs[0].mask.device
        self.device = dev
        self.results: list[RunResult] = []
        self.summaries, self.depths = [], []
        self.c_bins = None
        arr = (McJob * len(jobs))()
        for i, j in enumerate(jobs):
            vol = volume(j.mask)
            if accumulate_into is None:
                r = RunResult(torch.empty(tuple(j.mask.shape), dtype=torch.int64, device=dev),
                              torch.empty(NSCALARS, dtype=torch.int64, device=dev))
            else:
                r = accumulate_into.results[i]
            q = torch.empty(NSUMMARY, dtype=torch.float64, device=dev) if j.reduce else None
            d = torch.empty((3, j.mask.shape[0]), dtype=torch.float64, device=dev) if j.reduce else None
            self.results.append(r)
            self.summaries.append(q)
            self.depths.append(d)
            arr[i] = McJob(vol, j.optics.c(), j.photon_begin, j.n_photons, j.seed, j.stream_id,
                           1 if accumulate_into is not None else 0, r.fluence.data_ptr(), r.scalars.data_ptr(),
                           q.data_ptr() if q is not None else None, d.data_ptr() if d is not None else None)
        self.c_jobs = arr
        L = load()
        nbytes = L.mc_batch_workspace_bytes(ctypes.byref(arr), len(jobs))
        if nbytes == 0:
            raise McError(-1, "mc_batch_workspace_bytes", "invalid batch")
        self.ws = workspace(nbytes, dev)

    def attach_escape_bins(self, escape_bins: list, accumulate_into: "Batch | None" = None):
        """Per-job escape-path histograms: escape_bins[i] = (bin_width, nbins) or None.
        The tensors land in self.results[i].escape_hist_w / escape_hist_n."""
        if len(escape_bins) != len(self.jobs):
            raise ValueError("escape_bins needs one entry (or None) per job")
        arr = (McEscapeBins * len(self.jobs))()
        for i, eb in enumerate(escape_bins):
            r = self.results[i]
            if eb is None:
                arr[i] = McEscapeBins(1.0, 1, 0, None, None)
                continue
            width, nbins = float(eb[0]), int(eb[1])
            if accumulate_into is not None:
                if r.escape_hist_w is None or r.escape_hist_w.numel() != nbins:
                    raise ValueError(f"job {i}: accumulate needs a result that carries histograms of the same nbins")
            else:
                r.escape_hist_w = torch.empty(max(nbins, 1), dtype=torch.int64, device=self.device)
                r.escape_hist_n = torch.empty(max(nbins, 1), dtype=torch.int64, device=self.device)
            arr[i] = McEscapeBins(width, nbins, 0, r.escape_hist_w.data_ptr(), r.escape_hist_n.data_ptr())
        self.c_bins = arr

    def summary(self, i: int) -> Summary:
        q = self.summaries[i].cpu().numpy()
        d = self.depths[i].cpu().numpy()
        vals = {name: float(q[k]) for k, name in enumerate(SUMMARY)}
        _summary_status(vals["status"], f"mc_run_batch job {i}")
        return Summary(vals, d[0], d[1], d[2])


def run_batch(jobs: list[BatchJob], tune: Tune | None = None, fp64: bool = False, timed: bool = False,
              accumulate_into: Batch | None = None, escape_bins: list | None = None,
              line_staging: bool = False) -> Batch:
    """mc_run_batch on the current stream; tune None: the cached (or autotuned) launch shape.
    escape_bins: one (bin_width, nbins) or None per job: mc_run_batch_escape_histogram,
    which also bins each job's escaping photons by in-pore path into
    batch.results[i].escape_hist_w / escape_hist_n.  line_staging: MC_LINE_STAGING."""
    L = load()
    b = Batch(jobs, accumulate_into)
    flags = (MC_FP64 if fp64 else 0) | (MC_TIMED if timed else 0) | (MC_LINE_STAGING if line_staging else 0)
    t = tune.c() if tune is not None else None
    tref = ctypes.byref(t) if t is not None else None
    if escape_bins is None:
        _check(L.mc_run_batch(ctypes.byref(b.c_jobs), len(jobs), flags, tref, b.ws.data_ptr(), b.ws.numel(),
                              _stream(b.device)), "mc_run_batch")
    else:
        b.attach_escape_bins(escape_bins, accumulate_into)
        _check(L.mc_run_batch_escape_histogram(ctypes.byref(b.c_jobs), len(jobs), flags, tref,
                                               ctypes.byref(b.c_bins), b.ws.data_ptr(), b.ws.numel(),
                                               _stream(b.device)), "mc_run_batch_escape_histogram")
    if timed:
        ms = ctypes.c_float(0.0)
        _check(L.mc_walk_elapsed_ms(ctypes.byref(ms)), "mc_walk_elapsed_ms")
        b.walk_ms = float(ms.value)
    return b


def autotune_batch(jobs: list[BatchJob], fp64: bool = False) -> Tune:
    L = load()
    b = Batch(jobs)
    out = McTune()
    _check(L.mc_autotune_batch(ctypes.byref(b.c_jobs), len(jobs), MC_FP64 if fp64 else 0, b.ws.data_ptr(),
                               b.ws.numel(), ctypes.byref(out), _stream(b.device)), "mc_autotune_batch")
    return Tune(out.block, out.waves_per_cu, out.chunk, out.refill, out.defer)


class BatchGraph:
    """A captured HIP graph of one batched step; replay with launch()."""

    def __init__(self, jobs: list[BatchJob], tune: Tune | None = None, fp64: bool = False):
        L = load()
        self.batch = Batch(jobs)
        self.handle = ctypes.c_void_p()
        t = tune.c() if tune is not None else None
        _check(L.mc_batch_graph_create(ctypes.byref(self.batch.c_jobs), len(jobs), MC_FP64 if fp64 else 0,
                                       ctypes.byref(t) if t is not None else None, self.batch.ws.data_ptr(),
                                       self.batch.ws.numel(), ctypes.byref(self.handle)), "mc_batch_graph_create")

    def launch(self):
        _check(load().mc_graph_launch(self.handle, _stream(self.batch.device)), "mc_graph_launch")

    def close(self):
        if self.handle:
            load().mc_graph_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class GradResult:
    """Forward tallies of the gradient walk, its raw score bins and the Jacobian."""
    run: RunResult
    bins: torch.Tensor            # int64 [3, 2, nz, 2] (hi, lo)
    jac: torch.Tensor             # float64 [3, 2 + nz]
    summary: torch.Tensor         # float64 [NSUMMARY]
    depth: torch.Tensor           # float64 [3, nz]

    def bins_value(self) -> np.ndarray:
        """Exact bin values (hi * 2^32 + lo) as float64 [3, 2, nz], units 2^-GRAD_FIXED_BITS Q31 weight x voxel."""
        b = self.bins.cpu().numpy()
        hi = b[..., 0].astype(np.float64)
        lo = b[..., 1].view(np.uint64).astype(np.float64)
        return hi * 4294967296.0 + lo


def grad(mask: torch.Tensor, optics: Optics, n_photons: int, seed: int, photon_begin: int = 0, stream_id: int = 0,
         fp64: bool = False, timed: bool = False, tune: Tune | None = None, line_staging: bool = False) -> GradResult:
    """mc_grad on the current stream (line_staging: MC_LINE_STAGING)."""
    L = load()
    vol = volume(mask)
    dev = mask.device
    nz = mask.shape[0]
    run_ = RunResult(torch.empty(tuple(mask.shape), dtype=torch.int64, device=dev),
                     torch.empty(NSCALARS, dtype=torch.int64, device=dev))
    bins = torch.empty((3, 2, nz, 2), dtype=torch.int64, device=dev)
    jac = torch.empty((3, 2 + nz), dtype=torch.float64, device=dev)
    summary = torch.empty(NSUMMARY, dtype=torch.float64, device=dev)
    depth = torch.empty((3, nz), dtype=torch.float64, device=dev)
    ws = workspace(L.mc_grad_workspace_bytes(ctypes.byref(vol)), dev)
    opt = optics.c()
    t = tune.c() if tune is not None else None
    flags = (MC_FP64 if fp64 else 0) | (MC_TIMED if timed else 0) | (MC_LINE_STAGING if line_staging else 0)
    _check(L.mc_grad(ctypes.byref(vol), ctypes.byref(opt), photon_begin, n_photons, seed, stream_id, flags,
                     run_.fluence.data_ptr(), run_.scalars.data_ptr(), bins.data_ptr(), jac.data_ptr(),
                     summary.data_ptr(), depth.data_ptr(), ws.data_ptr(), ws.numel(),
                     ctypes.byref(t) if t is not None else None, _stream(dev)), "mc_grad")
    res = GradResult(run_, bins, jac, summary, depth)
    res._ws = ws
    if timed:
        ms = ctypes.c_float(0.0)
        _check(L.mc_walk_elapsed_ms(ctypes.byref(ms)), "mc_walk_elapsed_ms")
        res.walk_ms = float(ms.value)
    return res


class PhiFn(torch.autograd.Function):
    """(mu_s, mu_a, g) -> (<Phi>_3D, <Phi>_1D, Phi(z)) through the HIP walk.

    forward: mc_run + mc_reduce.  backward: mc_grad replays the same photons
    (same seed, stream and ids) and returns the likelihood-ratio Jacobian, which is
    contracted with the incoming gradients.  The coefficients enter as float32.
    """

    @staticmethod
    def forward(ctx, mu_s, mu_a, g, mask, n_photons, seed, stream_id=0, fp64=False):
        base = Optics(float(mu_s), float(mu_a), float(g))
        r = run(mask, base, n_photons, seed, stream_id=stream_id, fp64=fp64)
        q, d, ws = reduce_async(mask, r)
        _summary_status(float(q[SUMMARY.index("status")].item()), "PhiFn")
        ctx.save_for_backward(mu_s, mu_a, g)
        ctx.cfg = (mask, base, n_photons, seed, stream_id, fp64)
        return (q[SUMMARY.index("phi3d")].clone(), q[SUMMARY.index("phi1d")].clone(), d[0].clone())

    @staticmethod
    def backward(ctx, g3, g1, gz):
        mask, base, n_photons, seed, stream_id, fp64 = ctx.cfg
        jac = grad(mask, base, n_photons, seed, stream_id=stream_id, fp64=fp64).jac     # [3, 2 + nz]
        v = torch.cat([g3.reshape(1), g1.reshape(1), gz.reshape(-1)]).to(jac.dtype)
        out = jac @ v
        mu_s, mu_a, g = ctx.saved_tensors
        return (out[0].to(mu_s.dtype), out[1].to(mu_a.dtype), out[2].to(g.dtype), None, None, None, None, None)


def rms_w(profile, reference, device="cuda:0") -> dict:
    """mc_rms_w (Sec. 2.7, Eq. RMSw, and Table S1's variants) of a depth profile
    against a reference, on the GPU: {"weighted", "unweighted", "log"}, fractions."""
    dev = torch.device(device)
    p = torch.as_tensor(np.asarray(profile.cpu() if torch.is_tensor(profile) else profile, dtype=np.float64),
                        device=dev).contiguous()
    q = torch.as_tensor(np.asarray(reference.cpu() if torch.is_tensor(reference) else reference, dtype=np.float64),
                        device=dev).contiguous()
    if p.shape != q.shape or p.dim() != 1:
        raise ValueError("profile and reference must be 1-D arrays of one length")
    out = torch.empty(3, dtype=torch.float64, device=dev)
    _check(load().mc_rms_w(p.data_ptr(), q.data_ptr(), int(p.numel()), out.data_ptr(), _stream(dev)), "mc_rms_w")
    w, u, lg = out.cpu().tolist()
    return {"weighted": w, "unweighted": u, "log": lg}
