"""ctypes binding of liblrbms.so (include/lrbms.h).

Argument marshalling only: every step of the online path runs in the HIP
kernels of the library.  Device buffers are torch tensors on the GPU (their
data_ptr is passed through), streams are torch streams (their raw hipStream_t).
The library must be built (``python -m paper_1405_2810_amd.build`` or
``__graft_entry__.build()``); importing this module without it fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrbms.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lrbms.h")

DIRECT, DIRECT_FIT, AFFINE = 0, 1, 2
ERRORS = {0: "OK", -1: "E_ARG", -2: "E_STATE", -3: "E_OOM", -4: "E_HIP", -5: "E_NOT_SPD",
          -6: "E_NONFINITE", -7: "E_ADMIT"}


class LrbmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Problem_C(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("len", C.c_double * 3),
                ("nc", C.c_int32 * 3), ("cuts", C.c_void_p * 3),
                ("perm", C.c_void_p), ("poro", C.c_void_p),
                ("visc_w", C.c_double), ("visc_o", C.c_double),
                ("relperm", C.c_int32), ("corey_w", C.c_double), ("corey_o", C.c_double),
                ("bc_type", C.c_void_p), ("bc_val", C.c_void_p), ("bc_sat", C.c_void_p),
                ("bc_sval", C.c_void_p), ("q1", C.c_void_p), ("q2", C.c_void_p),
                ("penalty_c", C.c_double), ("weights", C.c_int32),
                ("sat_penalty_scale", C.c_double), ("limiter", C.c_int32), ("dt", C.c_double),
                ("dens_w", C.c_double), ("dens_o", C.c_double), ("grav", C.c_double * 3)]


class KernelStat_C(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


class ModelInfo_C(C.Structure):
    _fields_ = [("dim", C.c_int32), ("r", C.c_int32), ("ncell", C.c_int32), ("nface", C.c_int32),
                ("n_sub", C.c_int32), ("n_iface", C.c_int32), ("N", C.c_int32),
                ("n_profiles", C.c_int32), ("n_block_entries", C.c_int64),
                ("device_bytes", C.c_int64)]


class TuneReport_C(C.Structure):
    _fields_ = [("leaf_max", C.c_int32), ("split_min", C.c_int32), ("n_candidates", C.c_int32),
                ("bw_split_min", C.c_int32), ("us_per_solve", C.c_double),
                ("us_before", C.c_double), ("unrefined_error", C.c_double),
                ("refine", C.c_int32), ("asm_variant", C.c_int32), ("asm_us", C.c_double * 2)]


class OfflineOpts_C(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_train", C.c_int32), ("ne_cap", C.c_int32),
                ("unit_functions", C.c_int32), ("horizon", C.c_double), ("pcg_rtol", C.c_double),
                ("pcg_maxit", C.c_int32), ("tof_tol", C.c_double), ("tof_maxit", C.c_int32),
                ("keep_profiles", C.c_int32), ("d_s0", C.c_void_p), ("basis_method", C.c_int32),
                ("pca_eps", C.c_double)]


BASIS_METHODS = {"gs": 0, "pca": 1}   # LRBMS_BASIS_GS, LRBMS_BASIS_PCA


class OfflineReport_C(C.Structure):
    _fields_ = [("n_solves", C.c_int32), ("pcg_iters_max", C.c_int32),
                ("pcg_iters_total", C.c_int64), ("pcg_relres_max", C.c_double),
                ("tof_sweeps", C.c_int32), ("n_profiles_kept", C.c_int32)]


FIELD_SATURATION, FIELD_MOBILITY = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1405_2810_amd/build.py")
        # torch ships its own HIP runtime with the same soname as the system one;
        # loading torch first makes the library bind to that single runtime, so
        # device pointers and streams are shared with torch tensors.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.lrbms_last_error.restype = C.c_char_p
        L.lrbms_model_create.argtypes = [vp, vp, vp, i32, vp, C.POINTER(vp)]
        L.lrbms_model_create_from_snapshots.argtypes = [vp, i32, vp, i32, i32, i32, C.c_double,
                                                        i32, vp, C.POINTER(vp)]
        L.lrbms_model_get_info.argtypes = [vp, vp]
        L.lrbms_model_export_basis.argtypes = [vp, vp, vp]
        L.lrbms_model_interfaces.argtypes = [vp, vp, vp, vp]
        L.lrbms_online_assemble.argtypes = [vp, vp, i32, vp]
        L.lrbms_online_solve.argtypes = [vp, vp, vp]
        L.lrbms_model_set_refinement.argtypes = [vp, i32]
        L.lrbms_model_set_solver_shapes.argtypes = [vp, i32, i32, i32]
        L.lrbms_model_set_assembly_variant.argtypes = [vp, i32]
        L.lrbms_model_set_checks.argtypes = [vp, i32]
        L.lrbms_reconstruct_flux.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lrbms_transport_step.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lrbms_copy_reduced_system.argtypes = [vp, vp, vp]
        L.lrbms_copy_theta.argtypes = [vp, vp]
        L.lrbms_model_status.argtypes = [vp]
        L.lrbms_profile_enable.argtypes = [vp, i32]
        L.lrbms_profile_read.argtypes = [vp, vp, i32, C.POINTER(i32)]
        L.lrbms_build_offline_bases.argtypes = [vp, vp, vp, C.POINTER(vp), vp]
        L.lrbms_fine_pressure.argtypes = [vp, vp, i32, dbl, i32, vp, C.POINTER(i32),
                                          C.POINTER(dbl)]
        L.lrbms_time_of_flight.argtypes = [vp, vp, dbl, i32, vp, C.POINTER(i32)]
        L.lrbms_time_of_flight_noalloc.argtypes = [vp, vp, dbl, i32, vp, C.POINTER(i32)]
        L.lrbms_model_export_profiles.argtypes = [vp, vp]
        L.lrbms_build_greedy_bases.argtypes = [vp, vp, vp, i32, dbl, vp, C.POINTER(vp), vp, vp,
                                               i32, C.POINTER(i32), vp]
        L.lrbms_fine_create.argtypes = [vp, C.POINTER(vp)]
        L.lrbms_fine_step.argtypes = [vp, vp, dbl, i32, i32, vp, vp, vp, vp, C.POINTER(i32),
                                      C.POINTER(dbl)]
        L.lrbms_fine_destroy.argtypes = [vp]
        L.lrbms_fine_destroy.restype = None
        L.lrbms_model_destroy.argtypes = [vp]
        L.lrbms_model_destroy.restype = None
        L.lrbms_model_autotune.argtypes = [vp, vp, i32, vp]
        L.lrbms_batch_create.argtypes = [vp, i32, i32, i32, C.POINTER(vp)]
        L.lrbms_batch_step.argtypes = [vp, vp, vp, vp]
        L.lrbms_batch_buffers.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(vp)]
        L.lrbms_batch_status.argtypes = [vp]
        L.lrbms_batch_destroy.argtypes = [vp]
        L.lrbms_batch_destroy.restype = None
        L.lrbms_server_create.argtypes = [C.c_int64, i32, i32, C.POINTER(vp)]
        L.lrbms_server_attach.argtypes = [vp, vp, vp, C.POINTER(i32)]
        L.lrbms_server_submit.argtypes = [vp, i32, C.c_uint64]
        L.lrbms_server_poll.argtypes = [vp, vp, vp, vp, i32, C.POINTER(i32)]
        L.lrbms_server_drain.argtypes = [vp]
        L.lrbms_server_detach.argtypes = [vp, i32]
        L.lrbms_server_info.argtypes = [vp, vp]
        L.lrbms_server_set_fused.argtypes = [vp, i32]
        L.lrbms_server_destroy.argtypes = [vp]
        L.lrbms_server_destroy.restype = None
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions declared in include/lrbms.h."""
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(lrbms_\w+)\s*\(", src, re.M)))


def _check(rc):
    if rc < 0:
        raise LrbmsError(rc, lib().lrbms_last_error().decode())
    return rc


def _ptr(a) -> int:
    """Address of a numpy array or torch tensor (0 for None)."""
    if a is None:
        return 0
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _dev(t, dtype: str, n: int, name: str, optional: bool = False) -> int:
    """Device address of a caller buffer handed to device kernels: a
    contiguous torch tensor on the GPU of the expected dtype ("float64" or
    "uint8") with at least n elements; anything else raises LrbmsError(-1)
    (E_ARG) before any device work."""
    if t is None:
        if optional:
            return 0
        raise LrbmsError(-1, f"{name}: a device tensor is required")
    import torch
    want = {"float64": torch.float64, "uint8": torch.uint8}[dtype]
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise LrbmsError(-1, f"{name}: expected a torch tensor on the GPU")
    if t.dtype != want:
        raise LrbmsError(-1, f"{name}: expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise LrbmsError(-1, f"{name}: tensor must be contiguous")
    if t.numel() < n:
        raise LrbmsError(-1, f"{name}: {t.numel()} elements, {n} needed")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class ProblemC:
    """lrbms_problem built from any object with the fields of a problem
    description (dim, n, L, cuts, perm, poro, visc_w, ...).  Keeps the host
    arrays alive while the struct is in use."""

    def __init__(self, p):
        self._keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(np.asarray(x), dtype=dt)
            self._keep.append(a)
            return a.ctypes.data

        s = Problem_C()
        s.dim = int(p.dim)
        for a in range(3):
            s.n[a] = int(p.n[a]) if a < p.dim else 1
            s.len[a] = float(p.L[a]) if a < p.dim else 1.0
            s.nc[a] = (len(p.cuts[a]) - 1) if a < p.dim else 1
            s.cuts[a] = arr(p.cuts[a], np.int32) if a < p.dim else None
        s.perm, s.poro = arr(p.perm, np.float64), arr(p.poro, np.float64)
        s.visc_w, s.visc_o = float(p.visc_w), float(p.visc_o)
        s.relperm, s.corey_w, s.corey_o = int(p.relperm), float(p.corey_w), float(p.corey_o)
        s.bc_type, s.bc_val = arr(p.bc_type, np.int8), arr(p.bc_val, np.float64)
        s.bc_sat, s.bc_sval = arr(p.bc_sat, np.int8), arr(p.bc_sval, np.float64)
        s.q1, s.q2 = arr(p.q1, np.float64), arr(p.q2, np.float64)
        s.penalty_c, s.weights = float(p.penalty_c), int(p.weights)
        s.sat_penalty_scale, s.limiter, s.dt = float(p.sat_penalty_scale), int(p.limiter), float(p.dt)
        s.dens_w, s.dens_o = float(p.dens_w), float(p.dens_o)
        for a in range(3):
            s.grav[a] = float(p.grav[a])
        self.struct = s

    def ref(self):
        return C.byref(self.struct)


class Model:
    """An LRBMS model resident on the device (opaque lrbms_model handle)."""

    _owner = None   # the open Batch or Server holding the model, if any

    def __init__(self, handle, prob):
        self._h = handle
        self.prob = prob
        self._read_info()

    def _read_info(self):
        """lrbms_model_get_info; read again by every call that changes the
        model's device memory (solver shapes, assembly variant, autotune)."""
        info = ModelInfo_C()
        _check(lib().lrbms_model_get_info(self._h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in ModelInfo_C._fields_}

    # ---- creation ----------------------------------------------------
    @classmethod
    def create(cls, prob, sizes: Sequence[int], basis: np.ndarray, profiles=None):
        pc = ProblemC(prob)
        sz = np.ascontiguousarray(sizes, dtype=np.int32)
        bs = np.ascontiguousarray(basis, dtype=np.float64)
        prof = None if profiles is None or len(profiles) == 0 else \
            np.ascontiguousarray(np.stack(profiles), dtype=np.float64)
        h = C.c_void_p()
        _check(lib().lrbms_model_create(pc.ref(), _ptr(sz), _ptr(bs),
                                        0 if prof is None else prof.shape[0], _ptr(prof), C.byref(h)))
        m = cls(h, prob)
        m._sizes = sz.copy()
        m._offs = np.concatenate([[0], np.cumsum(sz)])
        return m

    @classmethod
    def from_snapshots(cls, prob, snapshots, ne_cap: int, unit_functions=True, profiles=None,
                       method: str = "gs", pca_eps: float = 1e-4):
        """Local bases from host snapshots by Gram-Schmidt or PCA on the device
        (lrbms_model_create_from_snapshots)."""
        pc = ProblemC(prob)
        sn = np.ascontiguousarray(np.stack(snapshots), dtype=np.float64)
        prof = None if profiles is None or len(profiles) == 0 else \
            np.ascontiguousarray(np.stack(profiles), dtype=np.float64)
        h = C.c_void_p()
        _check(lib().lrbms_model_create_from_snapshots(
            pc.ref(), sn.shape[0], _ptr(sn), int(ne_cap), int(bool(unit_functions)),
            BASIS_METHODS[method], float(pca_eps), 0 if prof is None else prof.shape[0],
            _ptr(prof), C.byref(h)))
        return cls(h, prob)

    @classmethod
    def build_offline(cls, prob, mu, ne_cap: int, horizon: float, unit_functions=True,
                      keep_profiles=True, pcg_rtol=1e-13, pcg_maxit=20000, tof_tol=1e-14,
                      tof_maxit=100000, s0=None, method: str = "gs", pca_eps: float = 1e-4):
        """Offline stage on the device (lrbms_build_offline_bases); mu is the
        (n_train, M) array of training parameters, s0 an optional device
        saturation whose flow defines the time of flight.  Returns (model,
        report)."""
        pc = ProblemC(prob)
        mu = np.ascontiguousarray(np.atleast_2d(mu), dtype=np.float64)
        o = OfflineOpts_C(M=mu.shape[1], n_train=mu.shape[0], ne_cap=int(ne_cap),
                          unit_functions=int(bool(unit_functions)), horizon=float(horizon),
                          pcg_rtol=float(pcg_rtol), pcg_maxit=int(pcg_maxit),
                          tof_tol=float(tof_tol), tof_maxit=int(tof_maxit),
                          keep_profiles=int(bool(keep_profiles)), d_s0=_ptr(s0) or None,
                          basis_method=BASIS_METHODS[method], pca_eps=float(pca_eps))
        rep = OfflineReport_C()
        h = C.c_void_p()
        _check(lib().lrbms_build_offline_bases(pc.ref(), C.byref(o), _ptr(mu), C.byref(h),
                                               C.byref(rep)))
        m = cls(h, prob)
        m._sizes = None
        return m, {f: getattr(rep, f) for f, _ in OfflineReport_C._fields_}

    @classmethod
    def build_greedy(cls, prob, mu, n_max: int, tol: float, horizon: float, mu_bar=None,
                     keep_profiles=True, pcg_rtol=1e-13, pcg_maxit=20000, tof_tol=1e-14,
                     tof_maxit=100000, s0=None):
        """Greedy basis construction on the device (lrbms_build_greedy_bases).
        Returns (model, chosen indices, error history, report)."""
        pc = ProblemC(prob)
        mu = np.ascontiguousarray(np.atleast_2d(mu), dtype=np.float64)
        o = OfflineOpts_C(M=mu.shape[1], n_train=mu.shape[0], ne_cap=1, unit_functions=0,
                          horizon=float(horizon), pcg_rtol=float(pcg_rtol),
                          pcg_maxit=int(pcg_maxit), tof_tol=float(tof_tol),
                          tof_maxit=int(tof_maxit), keep_profiles=int(bool(keep_profiles)),
                          d_s0=_ptr(s0) or None)
        mb = None if mu_bar is None else np.ascontiguousarray(mu_bar, dtype=np.float64)
        cap = 64
        chosen = np.full(cap, -1, dtype=np.int32)
        errs = np.zeros(cap)
        n = C.c_int32(0)
        rep = OfflineReport_C()
        h = C.c_void_p()
        _check(lib().lrbms_build_greedy_bases(pc.ref(), C.byref(o), _ptr(mu), int(n_max),
                                              float(tol), _ptr(mb), C.byref(h), _ptr(chosen),
                                              _ptr(errs), cap, C.byref(n), C.byref(rep)))
        m = cls(h, prob)
        m._sizes = None
        k = n.value
        return (m, [int(c) for c in chosen[:k] if c >= 0], errs[:k].tolist(),
                {f: getattr(rep, f) for f, _ in OfflineReport_C._fields_})

    def export_profiles(self) -> np.ndarray:
        out = np.empty((self.info["n_profiles"], self.info["r"] * self.info["ncell"]))
        _check(lib().lrbms_model_export_profiles(self._h, _ptr(out)))
        return out

    def close(self):
        """Destroy the model.  The library keeps a model that an open batch or
        server holds (it cannot be destroyed before them): close that first."""
        if self._h:
            if self._owner is not None and getattr(self._owner, "_h", None):
                raise LrbmsError(-2, "the model belongs to an open batch or server; "
                                     "close that first")
            lib().lrbms_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- online step --------------------------------------------------
    def _nsat(self):
        return self.info["r"] * self.info["ncell"]

    def assemble(self, sat, mode=DIRECT, stream=None):
        return _check(lib().lrbms_online_assemble(
            self._h, _dev(sat, "float64", self._nsat(), "sat"), int(mode), _stream(stream)))

    def solve(self, pN, stream=None):
        return _check(lib().lrbms_online_solve(self._h, _dev(pN, "float64", self.info["N"], "pN"),
                                               _stream(stream)))

    def set_refinement(self, steps: int):
        _check(lib().lrbms_model_set_refinement(self._h, int(steps)))

    def set_checks(self, on: bool):
        _check(lib().lrbms_model_set_checks(self._h, int(bool(on))))

    def reconstruct_flux(self, pN, sat, flux, ph=None, stream=None):
        n = self._nsat()
        return _check(lib().lrbms_reconstruct_flux(
            self._h, _dev(pN, "float64", self.info["N"], "pN"), _dev(sat, "float64", n, "sat"),
            _dev(flux, "float64", self.info["nface"], "flux"),
            _dev(ph, "float64", n, "ph", optional=True), _stream(stream)))

    def transport_step(self, sat, flux, sat_out, flags=None, stream=None):
        n = self._nsat()
        return _check(lib().lrbms_transport_step(
            self._h, _dev(sat, "float64", n, "sat"),
            _dev(flux, "float64", self.info["nface"], "flux"),
            _dev(sat_out, "float64", n, "sat_out"),
            _dev(flags, "uint8", self.info["ncell"], "flags", optional=True), _stream(stream)))

    # ---- inspection ---------------------------------------------------
    def reduced_system(self):
        blocks = np.empty(self.info["n_block_entries"])
        f = np.empty(self.info["N"])
        _check(lib().lrbms_copy_reduced_system(self._h, _ptr(blocks), _ptr(f)))
        return blocks, f

    def theta(self):
        t = np.empty(self.info["n_profiles"])
        _check(lib().lrbms_copy_theta(self._h, _ptr(t)))
        return t

    def interfaces(self):
        n = self.info["n_iface"]
        ax, lo, hi = (np.empty(n, dtype=np.int32) for _ in range(3))
        _check(lib().lrbms_model_interfaces(self._h, _ptr(ax), _ptr(lo), _ptr(hi)))
        return ax, lo, hi

    def box_cells(self) -> list:
        """Cells per coarse box, boxes in lexicographic order (x fastest)."""
        cuts = [np.asarray(c) for c in self.prob.cuts]
        out = []
        for ez in range(len(cuts[2]) - 1 if self.prob.dim == 3 else 1):
            for ey in range(len(cuts[1]) - 1):
                for ex in range(len(cuts[0]) - 1):
                    nz = (cuts[2][ez + 1] - cuts[2][ez]) if self.prob.dim == 3 else 1
                    out.append(int((cuts[0][ex + 1] - cuts[0][ex]) *
                                   (cuts[1][ey + 1] - cuts[1][ey]) * nz))
        return out

    def truncated(self, caps):
        """A new model with the first min(caps[E], N_E) basis functions of
        every box E (orthonormal subsets of the orthonormal local bases)."""
        sizes, flat = self.export_basis()
        r = self.info["r"]
        keep, parts, off = [], [], 0
        for NE, nE, cap in zip(sizes, self.box_cells(), caps):
            k = int(min(NE, cap))
            parts.append(flat[off:off + k * r * nE])
            keep.append(k)
            off += int(NE) * r * nE
        return Model.create(self.prob, keep, np.concatenate(parts))

    def export_basis(self):
        """(sizes, basis) as given to lrbms_model_create."""
        ncells = self.box_cells()
        sizes = np.empty(self.info["n_sub"], dtype=np.int32)
        basis = np.empty(sum(63 * self.info["r"] * n for n in ncells))   # at most 63 per box
        _check(lib().lrbms_model_export_basis(self._h, _ptr(sizes), _ptr(basis)))
        total = sum(int(k) * self.info["r"] * n for k, n in zip(sizes, ncells))
        return sizes, basis[:total].copy()

    def set_solver_shapes(self, leaf_max: int, split_min: int, bw_split_min: int):
        """Install the solver plan of given shapes (as a tune report gives
        them; 0 = never split) without timing (lrbms_model_set_solver_shapes)."""
        _check(lib().lrbms_model_set_solver_shapes(self._h, int(leaf_max), int(split_min),
                                                   int(bw_split_min)))
        self._read_info()

    def set_assembly_variant(self, variant: int):
        """Box assembly variant 0 or 1 (lrbms_model_set_assembly_variant)."""
        _check(lib().lrbms_model_set_assembly_variant(self._h, int(variant)))
        self._read_info()

    def autotune(self, sat, reps: int = 10) -> dict:
        """Time both box-assembly variants and every solver shape on the
        reduced system of `sat` and keep the fastest (lrbms_model_autotune)."""
        rep = TuneReport_C()
        _check(lib().lrbms_model_autotune(self._h, _ptr(sat), int(reps), C.byref(rep)))
        self._read_info()
        out = {k: getattr(rep, k) for k, _ in TuneReport_C._fields_}
        out["asm_us"] = list(rep.asm_us)
        return out

    def profile_enable(self, on: bool = True):
        """Switch the per-kernel event timing of the online calls on or off
        (clears the counters)."""
        _check(lib().lrbms_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """Per kernel: launches, summed device ms, algorithmic flops and bytes."""
        arr = (KernelStat_C * 32)()
        n = C.c_int32(0)
        _check(lib().lrbms_profile_read(self._h, C.cast(arr, C.c_void_p), 32, C.byref(n)))
        out = {}
        for k in range(min(n.value, 32)):
            e = arr[k]
            out[e.name.decode()] = {"launches": int(e.launches), "total_ms": float(e.total_ms),
                                    "flops": float(e.flops), "bytes": float(e.bytes)}
        return out

    def status(self):
        return lib().lrbms_model_status(self._h)

    def dense_reduced_matrix(self, blocks: Optional[np.ndarray] = None):
        """Scatter the block storage into a dense N x N matrix (host)."""
        if blocks is None:
            blocks, _ = self.reduced_system()
        sizes, offs = self.sizes_offsets()
        N = self.info["N"]
        A = np.zeros((N, N))
        pos = 0
        for E, ne in enumerate(sizes):
            A[offs[E]:offs[E] + ne, offs[E]:offs[E] + ne] = blocks[pos:pos + ne * ne].reshape(ne, ne)
            pos += ne * ne
        ax, lo, hi = self.interfaces()
        for t in range(len(ax)):
            nl, nh = sizes[lo[t]], sizes[hi[t]]
            B = blocks[pos:pos + nl * nh].reshape(nl, nh)
            A[offs[lo[t]]:offs[lo[t]] + nl, offs[hi[t]]:offs[hi[t]] + nh] = B
            A[offs[hi[t]]:offs[hi[t]] + nh, offs[lo[t]]:offs[lo[t]] + nl] = B.T
            pos += nl * nh
        return A

    def sparse_reduced_matrix(self, blocks: Optional[np.ndarray] = None, lower: bool = False):
        """The block storage as a scipy.sparse CSR matrix (host), both
        triangles of the coupling blocks; lower: each diagonal block taken
        from its lower triangle (the symmetric matrix the solver factors)."""
        import scipy.sparse as sp
        if blocks is None:
            blocks, _ = self.reduced_system()
        sizes, offs = self.sizes_offsets()
        rows, cols, vals = [], [], []
        pos = 0
        for E, ne in enumerate(sizes):
            i, j = np.meshgrid(np.arange(ne), np.arange(ne), indexing="ij")
            rows.append(offs[E] + i.ravel()); cols.append(offs[E] + j.ravel())
            blk = blocks[pos:pos + ne * ne]
            if lower:
                b2 = blk.reshape(ne, ne)
                blk = (np.tril(b2) + np.tril(b2, -1).T).ravel()
            vals.append(blk)
            pos += ne * ne
        ax, lo, hi = self.interfaces()
        for t in range(len(ax)):
            nl, nh = sizes[lo[t]], sizes[hi[t]]
            i, j = np.meshgrid(np.arange(nl), np.arange(nh), indexing="ij")
            v = blocks[pos:pos + nl * nh]
            rows += [offs[lo[t]] + i.ravel(), offs[hi[t]] + j.ravel()]
            cols += [offs[hi[t]] + j.ravel(), offs[lo[t]] + i.ravel()]
            vals += [v, v]
            pos += nl * nh
        N = self.info["N"]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(N, N))

    def sizes_offsets(self):
        if not hasattr(self, "_sizes"):
            self._sizes, _ = self.export_basis()
            self._offs = np.concatenate([[0], np.cumsum(self._sizes)])
        return self._sizes, self._offs


def fine_pressure(prob, field, p_out, kind=FIELD_SATURATION, rtol=1e-13, maxit=20000):
    """Fine SWIP pressure (lrbms_fine_pressure) into the device buffer p_out;
    returns (iterations, relative residual)."""
    pc = ProblemC(prob)
    it, rr = C.c_int32(0), C.c_double(0.0)
    _check(lib().lrbms_fine_pressure(pc.ref(), _ptr(field), int(kind), float(rtol), int(maxit),
                                     _ptr(p_out), C.byref(it), C.byref(rr)))
    return it.value, rr.value


def time_of_flight(prob, flux, tau_out, tol=0.0, maxit=100000, noalloc=False):
    """Time of flight (lrbms_time_of_flight, or lrbms_time_of_flight_noalloc
    with its fixed work memory) into the device buffer tau_out; returns the
    number of sweeps."""
    pc = ProblemC(prob)
    sw = C.c_int32(0)
    r, nface = int(prob.dim) + 1, len(prob.bc_type)
    ncell = int(np.prod(prob.n[:prob.dim]))
    fn = lib().lrbms_time_of_flight_noalloc if noalloc else lib().lrbms_time_of_flight
    _check(fn(pc.ref(), _dev(flux, "float64", nface, "flux"), float(tol), int(maxit),
              _dev(tau_out, "float64", r * ncell, "tau"), C.byref(sw)))
    return sw.value


class Fine:
    """Fine reference of Alg. 1 on the device (lrbms_fine handle)."""

    def __init__(self, prob):
        self.prob = prob
        self._h = C.c_void_p()
        _check(lib().lrbms_fine_create(ProblemC(prob).ref(), C.byref(self._h)))

    def step(self, sat, ph, flux, sat_out, flags=None, rtol=1e-13, maxit=20000, warm=False):
        """One time step; returns (CG iterations, relative residual)."""
        it, rr = C.c_int32(0), C.c_double(0.0)
        _check(lib().lrbms_fine_step(self._h, _ptr(sat), float(rtol), int(maxit), int(bool(warm)),
                                     _ptr(ph), _ptr(flux), _ptr(sat_out), _ptr(flags),
                                     C.byref(it), C.byref(rr)))
        return it.value, rr.value

    def close(self):
        if self._h:
            lib().lrbms_fine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solver_plan(prob, sizes, leaf_max: int = 2) -> dict:
    """Host-only export of the reduced solver's symbolic analysis
    (lrbms_solver_plan_export), parsed into Python structures."""
    L = lib()
    L.lrbms_solver_plan_export.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                           C.c_int64, C.c_void_p]
    pc = ProblemC(prob)
    sz = np.ascontiguousarray(sizes, dtype=np.int32)
    need = np.zeros(1, dtype=np.int64)
    _check(L.lrbms_solver_plan_export(pc.ref(), _ptr(sz), int(leaf_max), None, 0, _ptr(need)))
    buf = np.zeros(int(need[0]), dtype=np.int64)
    _check(L.lrbms_solver_plan_export(pc.ref(), _ptr(sz), int(leaf_max), _ptr(buf), buf.size,
                                      _ptr(need)))
    return _parse_plan(buf)


def solver_plan_batch(probs, sizes, leaf_max) -> dict:
    """Host-only export of the combined plan of a fused batch
    (lrbms_solver_plan_export_batch), parsed like solver_plan."""
    L = lib()
    L.lrbms_solver_plan_export_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                                 C.c_void_p, C.c_int64, C.c_void_p]
    n = len(probs)
    pcs = [ProblemC(p) for p in probs]
    szs = [np.ascontiguousarray(s, dtype=np.int32) for s in sizes]
    pp = (C.c_void_p * n)(*[C.addressof(pc.struct) for pc in pcs])
    sp = (C.c_void_p * n)(*[_ptr(s) for s in szs])
    lv = np.ascontiguousarray(leaf_max, dtype=np.int32)
    need = np.zeros(1, dtype=np.int64)
    _check(L.lrbms_solver_plan_export_batch(pp, sp, _ptr(lv), n, None, 0, _ptr(need)))
    buf = np.zeros(int(need[0]), dtype=np.int64)
    _check(L.lrbms_solver_plan_export_batch(pp, sp, _ptr(lv), n, _ptr(buf), buf.size, _ptr(need)))
    return _parse_plan(buf)


def _parse_plan(buf) -> dict:
    """Layout of the int64 plan record: a header (fronts, levels, nodes,
    children, L-store / front / vector / inverse doubles, flops); 12 values
    per front (off, voff, inv_off, m, u, node_off, n_nodes, child_off, nchild,
    n_s_nodes, npanels, loff); 4 per node reference (pos, pn_off, size, ppos);
    the children; per level its fronts, its extend-add items (7 values and
    three sources of 4) and its panel steps (items of 4: front, panel, ti, tj;
    a split step lists its rows-only items, then its update items); then the
    split backward products: partial-vector doubles, the U-row map, 3 values
    per front (nzc, urow_off, zoff) and per level its (front, chunk) items;
    then per level the (front, ti, tj, wide) tiles of the deferred Schur
    complements."""
    it = iter(buf.tolist())
    nxt = lambda k: [next(it) for _ in range(k)]
    nf, H, nn, nch, lpd, fd, vd, idd, flops = nxt(9)
    fronts = [dict(zip(["off", "voff", "inv_off", "m", "u", "node_off", "n_nodes", "child_off",
                        "nchild", "n_s_nodes", "npanels", "loff"], nxt(12))) for _ in range(nf)]
    nodes = [dict(zip(["pos", "pn_off", "size", "ppos"], nxt(4))) for _ in range(nn)]
    children = nxt(nch)
    levels = []
    for _ in range(H):
        lf = nxt(next(it))
        asm = []
        for _ in range(next(it)):
            d = dict(zip(["front", "dr", "dc", "nr", "nc", "diag", "nsrc"], nxt(7)))
            d["src"] = [dict(zip(["so", "rs", "cs", "kind"], nxt(4))) for _ in range(3)][:d["nsrc"]]
            asm.append(d)
        steps = []
        for _ in range(next(it)):
            steps.append([dict(zip(["front", "panel", "ti", "tj"], nxt(4))) for _ in range(next(it))])
        levels.append(dict(fronts=lf, asm=asm, steps=steps))
    # split backward products: partial storage, U-row map, per-front split
    # data (nzc chunks of 64 U rows, their first map entry, partial offset),
    # per-level work items (front, chunk)
    part = next(it)
    urow = nxt(next(it))
    for f in fronts:
        f["nzc"], f["urow_off"], f["zoff"] = nxt(3)
    for lev in levels:
        lev["bw"] = [tuple(nxt(2)) for _ in range(next(it))]
    # deferred Schur complements: per level (front, ti, tj, wide) output tiles
    for lev in levels:
        lev["schur"] = [tuple(nxt(4)) for _ in range(next(it))]
    if next(it, None) is not None:
        raise ValueError("plan record longer than its layout")
    return dict(fronts=fronts, nodes=nodes, children=children, levels=levels,
                front_doubles=fd, vec_doubles=vd, inv_doubles=idd, lpan_doubles=lpd, flops=flops,
                urow_pn=urow, bw_part_doubles=part)


BATCH_GRAPH = 1
BATCH_FUSED_SOLVE = 2


class ServerInfo_C(C.Structure):
    _fields_ = [("resident_bytes", C.c_int64), ("budget_bytes", C.c_int64),
                ("n_pending", C.c_int32), ("n_in_flight", C.c_int32),
                ("n_admitted", C.c_int32), ("n_waiting", C.c_int32)]


class Batch:
    """Batched ensemble (lrbms_batch_*): one time step of every model per
    ``step``; states are device tensors advanced in place.  Close it before
    closing its models."""

    def __init__(self, models: Sequence["Model"], mode=DIRECT, graph: bool = True,
                 fused: bool = False):
        self.models = list(models)
        arr = (C.c_void_p * len(self.models))(*[m._h for m in self.models])
        h = C.c_void_p()
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_FUSED_SOLVE if fused else 0)
        _check(lib().lrbms_batch_create(arr, len(self.models), mode, flags, C.byref(h)))
        self._h = h
        for m in self.models:
            m._owner = self

    def status(self) -> int:
        """Synchronize; first non-zero device status of the batch, else 0."""
        return lib().lrbms_batch_status(self._h)

    def step(self, sats, flags=None, stream=None):
        n = len(self.models)
        if len(sats) != n or (flags is not None and len(flags) != n):
            raise ValueError("one state (and flag buffer) per model")
        sp = (C.c_void_p * n)(*[_ptr(x) for x in sats])
        fp = None if flags is None else (C.c_void_p * n)(*[_ptr(x) for x in flags])
        _check(lib().lrbms_batch_step(self._h, sp, fp, _stream(stream)))

    def buffers(self, i: int):
        """Device addresses of simulation i's p_N and face fluxes."""
        a, b = C.c_void_p(), C.c_void_p()
        _check(lib().lrbms_batch_buffers(self._h, i, C.byref(a), C.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().lrbms_batch_destroy(self._h)
            self._h = None
            for m in self.models:
                if m._owner is self:
                    m._owner = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (lrbms_server_*): simulations attached with their state,
    admitted by memory footprint; requests (one time step each) dispatched
    onto slot streams as slots free up.  Close it before closing its models."""

    def __init__(self, hbm_budget: int, max_slots: int = 8, mode=DIRECT, fused: bool = False):
        self._carry = []
        self._sims = {}
        self._states = {}
        h = C.c_void_p()
        _check(lib().lrbms_server_create(int(hbm_budget), max_slots, mode, C.byref(h)))
        self._h = h
        if fused:
            _check(lib().lrbms_server_set_fused(self._h, 1))

    def attach(self, model: "Model", sat) -> int:
        """Attach a simulation with its state tensor; the server advances it
        in place and keeps a reference to it until detach or close."""
        sid = C.c_int32()
        ptr = _dev(sat, "float64", model.info["r"] * model.info["ncell"], "sat")
        _check(lib().lrbms_server_attach(self._h, model._h, ptr, C.byref(sid)))
        self._sims[sid.value] = model
        self._states[sid.value] = sat
        model._owner = self
        return sid.value

    def detach(self, sim: int):
        _check(lib().lrbms_server_detach(self._h, sim))
        self._states.pop(sim, None)
        m = self._sims.pop(sim, None)
        if m is not None and m._owner is self:
            m._owner = None

    def submit(self, sim: int, req_id: int):
        _check(lib().lrbms_server_submit(self._h, sim, req_id))

    def poll(self, cap: int = 256):
        """Finished requests, at most cap taken from the server per call: list
        of (req_id, latency_ms, status).  When the server reports an error
        after handing records over (its progress step failed), the records
        are kept and returned by the next call, and the error is raised."""
        ids = np.zeros(cap, np.uint64)
        lat = np.zeros(cap, np.float64)
        st = np.zeros(cap, np.int32)
        n = C.c_int32()
        rc = lib().lrbms_server_poll(self._h, ids.ctypes.data, lat.ctypes.data, st.ctypes.data,
                                     cap, C.byref(n))
        k = n.value
        got = self._carry + list(zip(ids[:k].tolist(), lat[:k].tolist(), st[:k].tolist()))
        self._carry = []
        if rc < 0:
            self._carry = got
            _check(rc)
        return got

    def drain(self):
        _check(lib().lrbms_server_drain(self._h))

    def info(self) -> dict:
        i = ServerInfo_C()
        _check(lib().lrbms_server_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in ServerInfo_C._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().lrbms_server_destroy(self._h)
            self._h = None
            for m in self._sims.values():
                if m._owner is self:
                    m._owner = None
            self._sims.clear()
            self._states.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
