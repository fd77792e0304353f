"""Thin ctypes binding of the C ABI in include/exx.h.

Argument marshalling only: every step of the pair-Poisson path runs in the
HIP kernels of libexx_mi355x.so.  There is no CPU fallback; if the library
is missing the import fails.  PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexx_mi355x.so")

EXX_OK, EXX_EINVAL, EXX_ENOMEM, EXX_EDEVICE, EXX_ENOCONV, EXX_ESTATE = 0, -1, -2, -3, -4, -5
_STATUS = {0: "EXX_OK", -1: "EXX_EINVAL", -2: "EXX_ENOMEM", -3: "EXX_EDEVICE", -4: "EXX_ENOCONV",
           -5: "EXX_ESTATE"}
PRECISION = {"fp64": 0, "fp32_refine": 1}
ORBITAL_DTYPE = {"f64": 0, "f32": 1}
GUESS = {"zero": 0, "previous": 1, "extrap": 2, "learned": 3}
PRECOND = {"none": 0, "mg": 1}
NLM = 49

EXPORTS = ["exx_default_params", "exx_setup", "exx_pairs", "exx_solve", "exx_energy_potential", "exx_stats",
           "exx_pair_info", "exx_debug_pair", "exx_last_error", "exx_destroy", "exx_model_init", "exx_model_train",
           "exx_model_save", "exx_load_model", "exx_model_edge", "exx_model_conv", "exx_model_wgrad",
           "exx_box_origins", "exx_pair_owners", "exx_pairs_spread",
           "exx_pair_class", "exx_stream_rates", "exx_solve_static"]


class ExxParams(C.Structure):
    _fields_ = [("n_grid", C.c_int32 * 3), ("cell", C.c_double * 3), ("r_pair", C.c_double),
                ("r_pe", C.c_double * 2), ("r_me", C.c_double * 2), ("fd_half_width", C.c_int32),
                ("l_max", C.c_int32), ("cg_rtol", C.c_double), ("cg_max_iter", C.c_int32),
                ("precision", C.c_int32), ("orbital_dtype", C.c_int32), ("guess", C.c_int32),
                ("inner_rtol", C.c_double), ("block_threads", C.c_int32), ("cg_cols", C.c_int32),
                ("wave_pairs", C.c_int64),
                ("keep_intermediates", C.c_int32), ("autotune", C.c_int32), ("graph", C.c_int32),
                ("box_dims", C.c_int32 * 3), ("precond", C.c_int32), ("n_classes", C.c_int32),
                ("class_r_pe", C.c_double * 4), ("class_r_me", C.c_double * 4), ("omega_scale", C.c_double)]


class ExxStats(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_self", C.c_int64), ("iters_total", C.c_int64),
                ("iters_min", C.c_int32), ("iters_max", C.c_int32), ("n_not_converged", C.c_int64),
                ("relres_max", C.c_double), ("solve_ms", C.c_double), ("prep_ms", C.c_double),
                ("cg_ms", C.c_double), ("dxx_ms", C.c_double), ("energy_ms", C.c_double),
                ("solve_grid", C.c_int32), ("solve_block", C.c_int32), ("cg_cols", C.c_int32),
                ("cg_bands", C.c_int32 * 2), ("outer_total", C.c_int64), ("n_pe", C.c_int64 * 2),
                ("n_me", C.c_int64 * 2), ("cg_bytes", C.c_int64), ("solve_bytes", C.c_int64),
                ("dxx_bytes", C.c_int64), ("device_bytes", C.c_int64), ("n_waves", C.c_int32), ("wave_n", C.c_int32),
                ("guess_pairs", C.c_int32), ("guess_ms", C.c_double), ("tuned", C.c_int32),
                ("tune_ms", C.c_double), ("graph_builds", C.c_int32), ("graph_launches", C.c_int32),
                ("n_classes", C.c_int32), ("class_n_pe", C.c_int64 * 4), ("class_n_me", C.c_int64 * 4),
                ("class_pairs", C.c_int64 * 4), ("class_capped", C.c_int64), ("cg_inflight", C.c_int32 * 2),
                ("cg_cols32", C.c_int32), ("cg_clock_ms", C.c_double)]


class ExxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1911_10630_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.exx_default_params.argtypes = [C.POINTER(ExxParams)]
    L.exx_default_params.restype = None
    L.exx_setup.argtypes = [C.POINTER(ExxParams), C.c_int, C.POINTER(vp)]
    L.exx_pairs.argtypes = [vp, i32, vp, C.POINTER(i64)]
    L.exx_solve.argtypes = [vp, vp, vp]
    L.exx_solve_static.argtypes = [vp, vp, vp]
    L.exx_solve_static.restype = C.c_int
    L.exx_energy_potential.argtypes = [vp, dp, vp, vp]
    L.exx_stats.argtypes = [vp, C.POINTER(ExxStats)]
    L.exx_pair_info.argtypes = [vp] + [vp] * 7
    L.exx_debug_pair.argtypes = [vp, i64] + [vp] * 5
    L.exx_last_error.argtypes = [vp]
    L.exx_last_error.restype = C.c_char_p
    L.exx_destroy.argtypes = [vp]
    L.exx_destroy.restype = None
    L.exx_box_origins.argtypes = [vp, vp]
    L.exx_pair_owners.argtypes = [vp, vp, vp]
    L.exx_pairs_spread.argtypes = [vp, i32, vp, vp, C.POINTER(i64)]
    L.exx_pair_class.argtypes = [vp, vp]
    L.exx_model_init.argtypes = [vp, i32, C.c_uint64]
    L.exx_model_train.argtypes = [vp, i32, i32, C.c_double, C.c_uint64, dp, vp]
    L.exx_model_save.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.exx_load_model.argtypes = [vp, vp, C.c_size_t]
    L.exx_model_edge.argtypes = [vp]
    L.exx_model_edge.restype = i32
    L.exx_model_conv.argtypes = [vp, i32, i32, vp, vp, i32, i32, vp]
    L.exx_model_wgrad.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp]
    L.exx_stream_rates.argtypes = [C.c_int, i64, i32, vp, vp, i32]
    L.exx_stream_rates.restype = C.c_int
    for f in ["exx_setup", "exx_pairs", "exx_solve", "exx_energy_potential", "exx_stats", "exx_pair_info",
              "exx_debug_pair", "exx_model_init", "exx_model_train", "exx_model_save", "exx_load_model",
              "exx_model_conv", "exx_model_wgrad", "exx_box_origins"]:
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def stream_rates(device: int = 0, bytes_per_array: int = 1 << 31, reps: int = 2) -> dict:
    """Measured streaming rates (GB/s) of plain read / copy / triad / cg-mix
    kernels on one device (exx_stream_rates)."""
    L = load()
    out = np.zeros(4)
    buf = C.create_string_buffer(512)
    st = L.exx_stream_rates(int(device), int(bytes_per_array), int(reps), _ptr(out), buf, 512)
    if st != EXX_OK:
        raise ExxError(st, "exx_stream_rates failed")
    return dict(read=float(out[0]), copy=float(out[1]), triad=float(out[2]), cg=float(out[3]),
                detail=buf.value.decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


class Exx:
    """One exact-exchange context on one GPU (exx_setup ... exx_destroy)."""

    def __init__(self, n_grid, cell, r_pair, r_pe, r_me, *, cg_rtol=1e-10, cg_max_iter=20000,
                 precision="fp64", orbital_dtype="f64", guess="zero", inner_rtol=1e-5, block_threads=0,
                 cg_cols=0, wave_pairs=0, keep_intermediates=False, autotune=True, graph=False, box=None, precond="none",
                 classes=None, omega_scale=0.0, device=0):
        L = load()
        p = ExxParams()
        L.exx_default_params(C.byref(p))
        for a in range(3):
            p.n_grid[a] = int(n_grid[a])
            p.cell[a] = float(cell[a])
        rpe = r_pe if isinstance(r_pe, (tuple, list)) else (r_pe, r_pe)
        rme = r_me if isinstance(r_me, (tuple, list)) else (r_me, r_me)
        p.r_pair = float(r_pair)
        p.r_pe[0], p.r_pe[1] = float(rpe[0]), float(rpe[1])
        p.r_me[0], p.r_me[1] = float(rme[0]), float(rme[1])
        p.cg_rtol = float(cg_rtol)
        p.cg_max_iter = int(cg_max_iter)
        p.precision = PRECISION[precision]
        p.orbital_dtype = ORBITAL_DTYPE[orbital_dtype]
        p.guess = GUESS[guess]
        p.inner_rtol = float(inner_rtol)
        p.block_threads = int(block_threads)
        p.cg_cols = int(cg_cols)
        p.wave_pairs = int(wave_pairs)
        p.keep_intermediates = 1 if keep_intermediates else 0
        p.autotune = 1 if autotune else 0
        p.graph = 1 if graph else 0
        p.precond = PRECOND[precond]
        if classes is not None:
            # per-pair subdomain classes: [(r_pe, r_me), ...], r_pe ascending
            p.n_classes = len(classes)
            for k, (a, b) in enumerate(classes):
                p.class_r_pe[k], p.class_r_me[k] = float(a), float(b)
            p.omega_scale = float(omega_scale)
        if box is not None:
            for a in range(3):
                p.box_dims[a] = int(box[a])
        self.params = p
        self.device = int(device)
        self.n_grid = tuple(int(v) for v in n_grid)
        self.box = tuple(int(box[a]) if box is not None and box[a] > 0 else self.n_grid[a] for a in range(3))
        self.orbital_dtype = orbital_dtype
        h = C.c_void_p()
        st = L.exx_setup(C.byref(p), self.device, C.byref(h))
        if st != EXX_OK:
            raise ExxError(st, L.exx_last_error(None).decode())
        self._h = h
        self.n_pairs = 0
        self.n_orb = 0

    @classmethod
    def from_workload(cls, wl, **kw):
        kw.setdefault("cg_rtol", wl.cg_rtol)
        kw.setdefault("precision", wl.precision)
        kw.setdefault("orbital_dtype", wl.orbital_dtype)
        if getattr(wl, "box", None) is not None:
            kw.setdefault("box", wl.box)
        return cls(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, **kw)

    def _check(self, st):
        if st != EXX_OK:
            raise ExxError(st, load().exx_last_error(self._h).decode())

    def pairs(self, centers) -> int:
        c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1, 3))
        n = C.c_int64()
        self._check(load().exx_pairs(self._h, c.shape[0], _ptr(c), C.byref(n)))
        self.n_pairs = int(n.value)
        self.n_orb = c.shape[0]
        return self.n_pairs

    def pairs_spread(self, centers, spreads) -> int:
        """The pair list with per-pair classes from the orbitals' spreads (bohr)."""
        c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1, 3))
        sp = np.ascontiguousarray(np.asarray(spreads, dtype=np.float64).reshape(-1))
        n = C.c_int64()
        self._check(load().exx_pairs_spread(self._h, c.shape[0], _ptr(c), _ptr(sp), C.byref(n)))
        self.n_pairs = int(n.value)
        self.n_orb = c.shape[0]
        return self.n_pairs

    def _check_grid(self, t, name):
        import torch
        want = torch.float64 if self.orbital_dtype == "f64" else torch.float32
        bx, by, bz = self.box
        if not t.is_cuda or t.dtype != want or not t.is_contiguous() or tuple(t.shape) != (self.n_orb, bz, by, bx):
            raise ValueError(f"{name} must be a contiguous {want} CUDA tensor of shape {(self.n_orb, bz, by, bx)}")

    def box_origins(self) -> np.ndarray:
        """[n_orb][3] grid origins of the orbital boxes (zeros for whole-grid storage)."""
        out = np.zeros((self.n_orb, 3), np.int32)
        self._check(load().exx_box_origins(self._h, _ptr(out)))
        return out

    def solve(self, phi, stream=None):
        self._check_grid(phi, "phi")
        self._phi = phi
        self._check(load().exx_solve(self._h, _ptr(phi), _stream_handle(stream, phi.device)))

    def solve_static(self, phi, stream=None):
        """exx_solve_static: the solve with its CG work vectors in the library's
        fixed device scratch (nothing allocated during the call)."""
        self._check_grid(phi, "phi")
        self._phi = phi
        self._check(load().exx_solve_static(self._h, _ptr(phi), _stream_handle(stream, phi.device)))

    def energy_potential(self, dxx, stream=None, allow_noconv=False) -> float:
        self._check_grid(dxx, "dxx")
        e = C.c_double()
        st = load().exx_energy_potential(self._h, C.byref(e), _ptr(dxx), _stream_handle(stream, dxx.device))
        if st == EXX_ENOCONV and allow_noconv:
            return e.value
        self._check(st)
        return e.value

    def step(self, phi, dxx=None, stream=None):
        import torch
        if dxx is None:
            dxx = torch.empty_like(phi)
        self.solve(phi, stream)
        return self.energy_potential(dxx, stream), dxx

    def stats(self) -> dict:
        s = ExxStats()
        self._check(load().exx_stats(self._h, C.byref(s)))
        out = {}
        for name, _ in ExxStats._fields_:
            v = getattr(s, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out

    def pair_info(self, results=True) -> dict:
        n = self.n_pairs
        d = dict(i=np.zeros(n, np.int32), j=np.zeros(n, np.int32), origin=np.zeros((n, 3), np.int32))
        if results:
            d.update(e=np.zeros(n), iters=np.zeros(n, np.int32), converged=np.zeros(n, np.int32),
                     relres=np.zeros(n))
        self._check(load().exx_pair_info(self._h, _ptr(d["i"]), _ptr(d["j"]), _ptr(d["origin"]),
                                         _ptr(d.get("e")), _ptr(d.get("iters")), _ptr(d.get("converged")),
                                         _ptr(d.get("relres"))))
        return d

    def pair_class(self) -> np.ndarray:
        """Subdomain class of each pair in pair_info order."""
        out = np.zeros(self.n_pairs, np.int32)
        self._check(load().exx_pair_class(self._h, _ptr(out)))
        return out

    def pair_owners(self):
        """Alg. 1 owner (i or j) of each pair in pair_info order, and the sweep count."""
        out = np.zeros(self.n_pairs, np.int32)
        sw = np.zeros(1, np.int32)
        self._check(load().exx_pair_owners(self._h, _ptr(out), _ptr(sw)))
        return out, int(sw[0])

    def debug_pair(self, pair: int, n_pe: int, n_shell: int, intermediates: bool = False) -> dict:
        d = dict(x=np.zeros(n_pe), vsh=np.zeros(max(n_shell, 1)), Q=np.zeros(NLM))
        if intermediates:
            d.update(rho=np.zeros(n_pe), b=np.zeros(n_pe))
        self._check(load().exx_debug_pair(self._h, int(pair), _ptr(d["x"]), _ptr(d["vsh"]), _ptr(d["Q"]),
                                          _ptr(d.get("rho")), _ptr(d.get("b"))))
        d["vsh"] = d["vsh"][:n_shell]
        return d

    # ---- learned initial guess -------------------------------------------

    def model_init(self, coarsen: int = 2, seed: int = 0):
        self._check(load().exx_model_init(self._h, int(coarsen), int(seed)))

    def model_train(self, epochs: int = 1, batch: int = 8, lr: float = 1e-3, seed: int = 0, stream=None) -> float:
        import torch
        loss = C.c_double()
        self._check(load().exx_model_train(self._h, int(epochs), int(batch), float(lr), int(seed), C.byref(loss),
                                           _stream_handle(stream, torch.device("cuda", self.device))))
        return loss.value

    def model_loss(self, batch: int = 8, stream=None) -> float:
        """Masked squared error of the model on the last solve's pairs (no update)."""
        return self.model_train(epochs=0, batch=batch, lr=0.0, stream=stream)

    def model_save(self) -> bytes:
        n = C.c_size_t()
        self._check(load().exx_model_save(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(load().exx_model_save(self._h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def load_model(self, blob: bytes):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._check(load().exx_load_model(self._h, buf, len(blob)))

    def model_edge(self) -> int:
        return int(load().exx_model_edge(self._h))

    def model_conv(self, layer: int, x, y, n: int, edge: int, transposed: bool = False, stream=None):
        self._check(load().exx_model_conv(self._h, int(layer), 1 if transposed else 0, _ptr(x), _ptr(y), int(n),
                                          int(edge), _stream_handle(stream, x.device)))

    def model_wgrad(self, layer: int, x, dy, dw, n: int, edge: int, stream=None):
        self._check(load().exx_model_wgrad(self._h, int(layer), _ptr(x), _ptr(dy), _ptr(dw), int(n), int(edge),
                                           _stream_handle(stream, x.device)))

    def close(self):
        if getattr(self, "_h", None):
            load().exx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
