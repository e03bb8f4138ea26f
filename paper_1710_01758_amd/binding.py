"""Thin ctypes binding of libpics.so (argument marshalling only).

Every computation runs in the native library; this module converts Python
arguments to the C ABI of include/pics.h.  Device buffers are torch tensors on
a ROCm device (torch is used for device memory and streams only).  Loading
fails loudly if the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpics.so")

PICS_OK = 0
PICS_WARN_MAXIT = 1
PICS_WARN_FALLBACK = 2
PICS_ERR_INVALID, PICS_ERR_UNSUPPORTED, PICS_ERR_NONFINITE, PICS_ERR_BREAKDOWN = -1, -2, -3, -4
PICS_ERR_NOT_POSITIVE, PICS_ERR_HIP, PICS_ERR_STATE = -5, -6, -7
MASK_LINES, MASK_2D = 0, 1
WAVELET = {"none": 0, "haar": 1, "db4": 2}
PRECOND = {"none": 0, "jacobi": 1, "circulant": 2, "learned": 3}
TERM_DATA, TERM_TV, TERM_GAMMA, TERM_ALL, TERM_WAVELET_EXPLICIT = 1, 2, 4, 7, 8
OPT_POLL_CHUNK = 1
OPT_GRAPH_BUDGET = 2
OPT_COIL_GROUPS = 3
OPT_CONCURRENT_GROUPS = 4
OPT_COL_TILE = 5
OPT_GRAPH_FIRST_BUDGET = 6
TUNE_FORCE = 1
TUNE_NO_WRITE = 2
OPT3_XCHUNK = 1


class PicsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pics error {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("ncoils", ctypes.c_int32),
                ("mask_kind", ctypes.c_int32), ("wavelet", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("mu", ctypes.c_double), ("lam", ctypes.c_double), ("gam", ctypes.c_double)]


class Desc3(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("ncoils", ctypes.c_int32),
                ("mu", ctypes.c_double), ("lam", ctypes.c_double), ("gam", ctypes.c_double)]


_LIB = None


def signatures():
    """ctypes (restype, argtypes) of every function the C ABI exports."""
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pi32, pdbl, pi64 = ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(i64)
    return {
        "pics_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, ctypes.POINTER(Desc), vp, vp, vp]),
        "pics_destroy": (ctypes.c_int, [vp]),
        "pics_sizes": (ctypes.c_int, [vp, pi64, pi64, pi64]),
        "pics_reserve": (ctypes.c_int, [vp, i32]),
        "build_preconditioner": (ctypes.c_int, [vp, i32, vp, vp]),
        "apply_A": (ctypes.c_int, [vp, vp, vp, i32]),
        "apply_A_noalloc": (ctypes.c_int, [vp, vp, vp, i32, i32]),
        "apply_Minv": (ctypes.c_int, [vp, vp, vp]),
        "pics_fft2": (ctypes.c_int, [vp, vp, vp, i32]),
        "pics_wavelet": (ctypes.c_int, [vp, vp, vp, i32]),
        "pcg_solve": (ctypes.c_int, [vp, vp, vp, dbl, i32, pi32, pi32, pdbl, pi32]),
        "split_bregman_recon": (ctypes.c_int, [vp, vp, i32, i32, dbl, i32, pi32, vp, pi32]),
        "pics_set_option": (ctypes.c_int, [vp, i32, i64]),
        "pics_autotune": (ctypes.c_int, [vp, i32]),
        "pics_coil_compress": (ctypes.c_int, [vp, vp, i32, vp, vp, pdbl]),
        "pics_get_tuning": (ctypes.c_int, [vp, pi32, i32]),
        "pics_get_tuning_tiles": (ctypes.c_int, [vp, pi32, i32]),
        "pics_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "pics_last_error": (ctypes.c_char_p, [vp]),
        "pics_features": (ctypes.c_int, [vp, vp, vp]),
        "pics_probe_stats": (ctypes.c_int, [vp, vp, i32, vp, vp, vp]),
        "pics_net_create": (ctypes.c_int, [ctypes.POINTER(vp), i32, vp]),
        "pics_net_destroy": (ctypes.c_int, [vp]),
        "pics_net_param_count": (i64, []),
        "pics_net_set_params": (ctypes.c_int, [vp, vp]),
        "pics_net_get_params": (ctypes.c_int, [vp, vp]),
        "pics_net_get_grad": (ctypes.c_int, [vp, vp]),
        "pics_net_forward": (ctypes.c_int, [vp, i32, vp, vp, vp]),
        "pics_net_loss_grad": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, pdbl]),
        "pics_net_adam_step": (ctypes.c_int, [vp, ctypes.c_float]),
        "pics_net_correction": (ctypes.c_int, [vp, vp, vp, vp]),
        "pics3d_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(Desc3), vp, vp, vp]),
        "pics3d_destroy": (ctypes.c_int, [vp]),
        "pics3d_build_preconditioner": (ctypes.c_int, [vp, i32, vp]),
        "pics3d_apply_A": (ctypes.c_int, [vp, vp, vp]),
        "pics3d_rhs": (ctypes.c_int, [vp, vp, vp]),
        "pics3d_apply_Minv": (ctypes.c_int, [vp, vp, vp]),
        "pics3d_pcg_solve": (ctypes.c_int, [vp, vp, vp, dbl, i32, pi32, pdbl]),
        "pics3d_last_error": (ctypes.c_char_p, [vp]),
        "pics3d_set_option": (ctypes.c_int, [vp, i32, i32]),
        "pics3d_get_option": (ctypes.c_int, [vp, i32, pi32]),
    }


def library_path():
    import pathlib
    return pathlib.Path(LIB_PATH)


def lib(path: str = LIB_PATH):
    """Load libpics.so (raises if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1710_01758_amd.build`")
    L = ctypes.CDLL(path)
    sig = signatures()
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _i32(a: Optional[np.ndarray]):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Context:
    """A batch of slices sharing one stream.  `descs` are (m, n, ncoils,
    wavelet name, levels, mu, lambda, gamma) records; `sens` (complex64) and
    `masks` (uint8) are packed device tensors kept alive by this object."""

    def __init__(self, descs: Sequence[dict], sens, masks, stream=None):
        import torch
        self.L = lib()
        self.n = len(descs)
        arr = (Desc * self.n)()
        for i, d in enumerate(descs):
            arr[i] = Desc(int(d["m"]), int(d["n"]), int(d["ncoils"]), MASK_LINES if d.get("mask_kind", "lines") == "lines" else MASK_2D,
                          WAVELET[d.get("wavelet", "db4")], int(d.get("levels", 0)), float(d["mu"]),
                          float(d["lam"]), float(d["gam"]))
        self.descs = list(descs)
        self._keep = (sens, masks)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.L.pics_create(ctypes.byref(h), self.n, arr, _ptr(sens), _ptr(masks), ctypes.c_void_p(stream))
        if rc != PICS_OK:
            raise PicsError(rc, self.L.pics_status_string(rc).decode())
        self.h = h
        img, coil, mk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.L.pics_sizes(self.h, ctypes.byref(img), ctypes.byref(coil), ctypes.byref(mk))
        self.image_elems, self.coil_elems, self.mask_bytes = img.value, coil.value, mk.value

    # -- helpers
    def _check(self, rc: int, allow_warn: bool = True) -> int:
        if rc < 0 or (rc > 0 and not allow_warn):
            raise PicsError(rc, self.L.pics_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.L.pics_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: int, value: int):
        return self._check(self.L.pics_set_option(self.h, key, value))

    def reserve(self, max_solves: int):
        """Room for Split Bregman runs of up to max_solves solves (64 by default)."""
        return self._check(self.L.pics_reserve(self.h, int(max_solves)))

    def autotune(self, flags: int = 0):
        """Time the coil splits of the fused operator per size group and keep
        the fastest; returns the chosen split per group."""
        self._check(self.L.pics_autotune(self.h, flags))
        return self.tuning()

    def tuning(self):
        buf = (ctypes.c_int32 * 64)()
        ng = self._check(self.L.pics_get_tuning(self.h, buf, 64))
        return [int(buf[i]) for i in range(ng)]

    def tuning_tiles(self):
        """Column-tile width of the line-mask operator per size group."""
        buf = (ctypes.c_int32 * 64)()
        ng = self._check(self.L.pics_get_tuning_tiles(self.h, buf, 64))
        return [int(buf[i]) for i in range(ng)]

    # -- entry points (same names as the C ABI)
    def build_preconditioner(self, kind: str = "circulant", correction=None, khat=None) -> int:
        return self._check(self.L.build_preconditioner(self.h, PRECOND[kind], _ptr(correction), _ptr(khat)))

    def apply_A(self, x, y, terms: int = TERM_ALL) -> int:
        return self._check(self.L.apply_A(self.h, _ptr(x), _ptr(y), terms))

    def apply_A_noalloc(self, x, y, terms: int = TERM_ALL, coil_groups: int = 1) -> int:
        return self._check(self.L.apply_A_noalloc(self.h, _ptr(x), _ptr(y), terms, int(coil_groups)))

    def apply_Minv(self, r, z) -> int:
        return self._check(self.L.apply_Minv(self.h, _ptr(r), _ptr(z)))

    def fft2(self, x, out, inverse: bool = False) -> int:
        return self._check(self.L.pics_fft2(self.h, _ptr(x), _ptr(out), int(inverse)))

    def wavelet(self, x, out, inverse: bool = False) -> int:
        return self._check(self.L.pics_wavelet(self.h, _ptr(x), _ptr(out), int(inverse)))

    def pcg_solve(self, b, x, tol: float, maxit: int, maxit_per_slice=None):
        iters = np.zeros(self.n, np.int32)
        relres = np.zeros(self.n, np.float64)
        status = np.zeros(self.n, np.int32)
        mp = _i32(maxit_per_slice)
        rc = self.L.pcg_solve(self.h, _ptr(b), _ptr(x), float(tol), int(maxit), mp[1] if mp else None,
                              iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              relres.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(rc)
        return iters, relres, status, rc

    def split_bregman_recon(self, kspace, x_out, n_outer: int = 20, n_inner: int = 1, tol: float = 1e-3,
                            maxit: int = 1000, lock=None):
        iters = np.zeros((n_outer * n_inner, self.n), np.int32)
        lk = _i32(None if lock is None else np.asarray(lock).reshape(n_outer * n_inner, self.n))
        rc = self.L.split_bregman_recon(self.h, _ptr(kspace), n_outer, n_inner, float(tol), int(maxit),
                                        lk[1] if lk else None, _ptr(x_out),
                                        iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(rc)
        return iters, rc

    def coil_compress(self, kspace, nvirt: int, kspace_out, sens_out):
        """Compress every slice to its nvirt most dominant virtual coils;
        returns the eigenvalues (descending, concatenated per slice)."""
        eig = np.zeros(sum(int(d["ncoils"]) for d in self.descs), np.float64)
        self._check(self.L.pics_coil_compress(self.h, _ptr(kspace), int(nvirt), _ptr(kspace_out), _ptr(sens_out),
                                              eig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return eig

    def features(self, khat, out):
        """Feature planes [nslices][6][64][64] (float32 device tensor `out`)."""
        return self._check(self.L.pics_features(self.h, _ptr(khat), _ptr(out)))

    def probe_stats(self, probes, nprobes: int, G, H, Z):
        return self._check(self.L.pics_probe_stats(self.h, _ptr(probes), int(nprobes), _ptr(G), _ptr(H), _ptr(Z)))


class Net:
    """The spectrum-correction network of libpics (parameters on the device)."""

    def __init__(self, batch_max: int, stream=None):
        import torch
        self.L = lib()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        rc = self.L.pics_net_create(ctypes.byref(h), int(batch_max), ctypes.c_void_p(stream))
        if rc != PICS_OK:
            raise PicsError(rc, self.L.pics_status_string(rc).decode())
        self.h = h
        self.batch_max = batch_max
        self.count = int(self.L.pics_net_param_count())

    def close(self):
        if getattr(self, "h", None):
            self.L.pics_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc < 0:
            raise PicsError(rc, self.L.pics_status_string(rc).decode())
        return rc

    def set_params(self, theta: np.ndarray):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        assert t.size == self.count
        return self._check(self.L.pics_net_set_params(self.h, t.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self) -> np.ndarray:
        t = np.empty(self.count, np.float32)
        self._check(self.L.pics_net_get_params(self.h, t.ctypes.data_as(ctypes.c_void_p)))
        return t

    def get_grad(self) -> np.ndarray:
        t = np.empty(self.count, np.float32)
        self._check(self.L.pics_net_get_grad(self.h, t.ctypes.data_as(ctypes.c_void_p)))
        return t

    def forward(self, batch: int, features, out, index=None):
        return self._check(self.L.pics_net_forward(self.h, int(batch), _ptr(index), _ptr(features), _ptr(out)))

    def loss_grad(self, batch: int, index, features, k, G, H, Z) -> float:
        loss = ctypes.c_double()
        self._check(self.L.pics_net_loss_grad(self.h, int(batch), _ptr(index), _ptr(features), _ptr(k), _ptr(G),
                                              _ptr(H), _ptr(Z), ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr: float):
        return self._check(self.L.pics_net_adam_step(self.h, ctypes.c_float(lr)))

    def correction(self, ctx: "Context", features, out):
        return self._check(self.L.pics_net_correction(self.h, ctx.h, _ptr(features), _ptr(out)))


# ---------------------------------------------------------------------------
# packing of host arrays into the library's layouts (marshalling only)

def spec_desc(spec) -> dict:
    return dict(m=spec.m, n=spec.n, ncoils=spec.ncoils, mask_kind=spec.mask_kind, wavelet=spec.wavelet,
                levels=spec.levels if spec.wavelet != "none" else 0, mu=spec.mu, lam=spec.lam, gam=spec.gam)


def pack_images(arrs: Sequence[np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(a, np.complex64).ravel() for a in arrs])


def unpack_images(flat: np.ndarray, shapes: Sequence[tuple]) -> List[np.ndarray]:
    out, o = [], 0
    for (m, n) in shapes:
        out.append(flat[o:o + m * n].reshape(m, n))
        o += m * n
    return out


def pack_masks(masks: Sequence[np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(mk, np.uint8).ravel() for mk in masks])


def to_device(a: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def context_for(instances, device="cuda", stream=None):
    """Create a Context for a list of inputs.Instance; returns (ctx, kspace_dev)."""
    sens = to_device(pack_images([inst.sens for inst in instances]), device)
    masks = to_device(pack_masks([inst.mask for inst in instances]), device)
    ctx = Context([spec_desc(inst.spec) for inst in instances], sens, masks, stream)
    ksp = to_device(pack_images([inst.kspace for inst in instances]), device)
    return ctx, ksp


class Volume:
    """A 3D problem on libpics (volume [p][m][n], one context per volume)."""

    def __init__(self, spec, sens, mask, stream=None):
        import torch
        self.L = lib()
        self.spec = spec
        self._keep = (sens, mask)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        d = Desc3(spec.p, spec.m, spec.n, spec.ncoils, spec.mu, spec.lam, spec.gam)
        h = ctypes.c_void_p()
        rc = self.L.pics3d_create(ctypes.byref(h), ctypes.byref(d), _ptr(sens), _ptr(mask), ctypes.c_void_p(stream))
        if rc != PICS_OK:
            raise PicsError(rc, self.L.pics_status_string(rc).decode())
        self.h = h
        self.voxels = spec.p * spec.m * spec.n

    def _check(self, rc: int) -> int:
        if rc < 0:
            raise PicsError(rc, self.L.pics3d_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.L.pics3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_preconditioner(self, kind: str = "circulant", khat=None) -> int:
        return self._check(self.L.pics3d_build_preconditioner(self.h, PRECOND[kind], _ptr(khat)))

    def apply_A(self, x, y) -> int:
        return self._check(self.L.pics3d_apply_A(self.h, _ptr(x), _ptr(y)))

    def apply_Minv(self, r, z) -> int:
        return self._check(self.L.pics3d_apply_Minv(self.h, _ptr(r), _ptr(z)))

    def rhs(self, kspace, b) -> int:
        return self._check(self.L.pics3d_rhs(self.h, _ptr(kspace), _ptr(b)))

    def set_option(self, option: int, value: int) -> int:
        return self._check(self.L.pics3d_set_option(self.h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int32()
        self._check(self.L.pics3d_get_option(self.h, int(option), ctypes.byref(v)))
        return v.value

    def pcg_solve(self, b, x, tol: float, maxit: int):
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        rc = self._check(self.L.pics3d_pcg_solve(self.h, _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(it),
                                                 ctypes.byref(rel)))
        return it.value, rel.value, rc


def volume_for(inst, device="cuda", stream=None):
    """A Volume context and its k-space (device c64) for an inputs.VolumeInstance."""
    sens = to_device(np.asarray(inst.sens, np.complex64).ravel(), device)
    mask = to_device(np.asarray(inst.mask, np.uint8).ravel(), device)
    ksp = to_device(np.asarray(inst.kspace, np.complex64).ravel(), device)
    return Volume(inst.spec, sens, mask, stream), ksp
