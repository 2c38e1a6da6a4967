"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this module.  The HIP library never imports it.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import build as _build

_LIB = None

WEIGHTED, MEAN, BEST = 0, 1, 2


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("patch", C.c_int32 * 3),
        ("levels", C.c_int32),
        ("lambda_", C.c_int32),
        ("pm_iters", C.c_int32),
        ("n_jf", C.c_int32),
        ("jf_steps", C.c_int32 * 8),
        ("rho", C.c_double),
        ("em_max_iters", C.c_int32),
        ("em_tol", C.c_double),
        ("recon_mode", C.c_int32),
        ("seed", C.c_uint64),
        ("temporal_subsample", C.c_int32),
    ]


class AlignParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("iters", C.c_int32), ("tukey_c", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        # VIO_LIB: another build of the same sources (the sanitizer test)
        path = os.environ.get("VIO_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER
        u8p, i32p, i64p, f32p = P(C.c_uint8), P(C.c_int32), P(C.c_int64), P(C.c_float)
        L.vio_params_default.argtypes = [P(Params)]
        L.vio_create.argtypes = [P(C.c_void_p), P(Params), C.c_int32, C.c_int32, C.c_int32,
                                 u8p, u8p]
        L.vio_destroy.argtypes = [C.c_void_p]
        L.vio_destroy.restype = None
        L.vio_level_info.argtypes = [C.c_void_p, C.c_int32, i32p, i64p]
        L.vio_level_sets.argtypes = [C.c_void_p, C.c_int32, u8p, u8p, u8p]
        L.vio_get_state.argtypes = [C.c_void_p, C.c_int32, u8p, i32p, i32p, u8p]
        L.vio_set_state.argtypes = [C.c_void_p, C.c_int32, u8p, i32p, i32p, u8p]
        L.vio_patch_ssd.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, u8p, i32p]
        L.vio_patch_ssd.restype = C.c_int64
        L.vio_philox4x64_10.argtypes = [P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.vio_philox4x64_10.restype = None
        L.vio_draw_below.argtypes = [C.c_uint64, C.c_int64]
        L.vio_draw_below.restype = C.c_int64
        L.vio_rs_candidate.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_int32,
                                       C.c_uint64]
        L.vio_rs_candidate.restype = C.c_int64
        L.vio_onion_layer.argtypes = [C.c_void_p, u8p, C.c_int32, u8p, u8p, f32p, i64p]
        L.vio_nnf_search.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
        L.vio_nnf_search_set.argtypes = [C.c_void_p, C.c_int32, u8p, u8p, C.c_uint64]
        L.vio_reconstruct.argtypes = [C.c_void_p, C.c_int32, C.c_int32, f32p, i64p]
        L.vio_inpaint_level.argtypes = [C.c_void_p, C.c_int32, i32p]
        L.vio_onion_init.argtypes = [C.c_void_p, i32p]
        L.vio_transition.argtypes = [C.c_void_p, C.c_int32]
        L.vio_inpaint.argtypes = [C.c_void_p, u8p]
        L.vio_energy.argtypes = [C.c_void_p, C.c_int32]
        L.vio_energy.restype = C.c_int64
        L.vio_num_threads.argtypes = []
        f64p = P(C.c_double)
        L.vio_align_params_default.argtypes = [P(AlignParams)]
        L.vio_align_estimate.argtypes = [u8p, u8p, C.c_int32, C.c_int32, C.c_int32,
                                         P(AlignParams), f64p]
        L.vio_align_compose.argtypes = [f64p, C.c_int32, f64p]
        L.vio_affine_inverse.argtypes = [f64p, f64p]
        L.vio_align_warp.argtypes = [u8p, u8p, C.c_int32, C.c_int32, C.c_int32, f64p, u8p, u8p]
        L.vio_align_unwarp.argtypes = [u8p, u8p, u8p, C.c_int32, C.c_int32, C.c_int32, f64p, u8p]
        L.vio_set_reduction.argtypes = [C.c_void_p, C.c_int32, P(C.c_int16), C.c_int32]
        L.vio_features.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32)]
        L.vio_pca_moments.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(C.c_uint64),
                                      P(C.c_uint64), P(C.c_int64)]
        L.vio_closer_than_constant.argtypes = [u8p, C.c_int32, u8p, C.c_int32, C.c_int32,
                                               C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                               C.c_int32, P(C.c_uint64)]
        _LIB = L
    return _LIB


def _ptr(a, ct):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(ct))


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, np.uint64).copy()
    k = np.asarray(key, np.uint64).copy()
    o = np.zeros(4, np.uint64)
    lib().vio_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(o, C.c_uint64))
    return o


def draw_below(w, n):
    return int(lib().vio_draw_below(C.c_uint64(int(w)), int(n)))


def default_params(**kw) -> Params:
    p = Params()
    lib().vio_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "jf_steps":
            p.n_jf = len(v)
            for i, s in enumerate(v):
                p.jf_steps[i] = s
        elif k == "patch":
            for i, s in enumerate(v):
                p.patch[i] = s
        elif k == "lam":
            p.lambda_ = v
        else:
            setattr(p, k, v)
    return p


class OracleError(RuntimeError):
    def __init__(self, fn, st):
        super().__init__(f"{fn} returned {st}")
        self.status = st


def _check(fn, st):
    if st != 0:
        raise OracleError(fn, st)


class Oracle:
    """One clip in the CPU oracle."""

    def __init__(self, video: np.ndarray, mask: np.ndarray, params: Params | None = None,
                 reduce_dims: int = 0, reduce_samples: int = 65536, **kw):
        self.params = params if params is not None else default_params(**kw)
        T, H, W, _ = video.shape
        self.W, self.H, self.T = W, H, T
        v = np.ascontiguousarray(video, np.uint8)
        m = np.ascontiguousarray(mask, np.uint8)
        h = C.c_void_p()
        st = lib().vio_create(C.byref(h), C.byref(self.params), W, H, T, _ptr(v, C.c_uint8),
                              _ptr(m, C.c_uint8))
        _check("vio_create", st)
        self.h = h
        if reduce_dims:
            # every level gets the PCA basis of its own source patches
            for level in range(self.params.levels):
                self.set_reduction(level, self.pca_basis(level, reduce_dims, reduce_samples))

    def close(self):
        if getattr(self, "h", None):
            lib().vio_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    @property
    def levels(self):
        return self.params.levels

    def info(self, level):
        d = np.zeros(3, np.int32)
        c = np.zeros(3, np.int64)
        _check("vio_level_info", lib().vio_level_info(self.h, level, _ptr(d, C.c_int32),
                                                      _ptr(c, C.c_int64)))
        return tuple(int(x) for x in d), tuple(int(x) for x in c)

    def dims(self, level):
        return self.info(level)[0]

    def sets(self, level):
        W, H, T = self.dims(level)
        hole = np.zeros((T, H, W), np.uint8)
        dsrc = np.zeros((T, H, W), np.uint8)
        htil = np.zeros((T, H, W), np.uint8)
        _check("vio_level_sets", lib().vio_level_sets(self.h, level, _ptr(hole, C.c_uint8),
                                                      _ptr(dsrc, C.c_uint8),
                                                      _ptr(htil, C.c_uint8)))
        return hole, dsrc, htil

    def get_state(self, level):
        W, H, T = self.dims(level)
        rgbt = np.zeros((T, H, W, 5), np.uint8)
        cand = np.zeros((T, H, W), np.int32)
        dist = np.zeros((T, H, W), np.int32)
        nvox = np.zeros((T, H, W), np.uint8)
        _check("vio_get_state", lib().vio_get_state(self.h, level, _ptr(rgbt, C.c_uint8),
                                                    _ptr(cand, C.c_int32),
                                                    _ptr(dist, C.c_int32),
                                                    _ptr(nvox, C.c_uint8)))
        return rgbt, cand, dist, nvox

    def set_state(self, level, rgbt=None, cand=None, dist=None, nvox=None):
        def c(a, dt):
            return None if a is None else np.ascontiguousarray(a, dt)
        rgbt, cand, dist, nvox = (c(rgbt, np.uint8), c(cand, np.int32), c(dist, np.int32),
                                  c(nvox, np.uint8))
        _check("vio_set_state", lib().vio_set_state(self.h, level, _ptr(rgbt, C.c_uint8),
                                                    _ptr(cand, C.c_int32),
                                                    _ptr(dist, C.c_int32),
                                                    _ptr(nvox, C.c_uint8)))

    def patch_ssd(self, level, p, c, count_mask=None):
        n = C.c_int32(0)
        cm = None if count_mask is None else np.ascontiguousarray(count_mask, np.uint8)
        d = lib().vio_patch_ssd(self.h, level, int(p), int(c), _ptr(cm, C.c_uint8), C.byref(n))
        return int(d), int(n.value)

    def nnf_search(self, level, em_iter=0):
        _check("vio_nnf_search", lib().vio_nnf_search(self.h, level, em_iter))

    def nnf_search_set(self, level, target_mask, count_mask=None, step=0):
        tm = np.ascontiguousarray(target_mask, np.uint8)
        cm = None if count_mask is None else np.ascontiguousarray(count_mask, np.uint8)
        _check("vio_nnf_search_set", lib().vio_nnf_search_set(
            self.h, level, _ptr(tm, C.c_uint8), _ptr(cm, C.c_uint8), C.c_uint64(step)))

    def reconstruct(self, level, mode=WEIGHTED, want_out=True):
        (_, _, _), (nH, _, _) = self.info(level)
        out = np.zeros((nH, 5), np.float32) if want_out else None
        s = C.c_int64(0)
        _check("vio_reconstruct", lib().vio_reconstruct(self.h, level, mode,
                                                        _ptr(out, C.c_float), C.byref(s)))
        return out, int(s.value)

    def inpaint_level(self, level):
        k = C.c_int32(0)
        _check("vio_inpaint_level", lib().vio_inpaint_level(self.h, level, C.byref(k)))
        return int(k.value)

    def onion_init(self):
        k = C.c_int32(0)
        _check("vio_onion_init", lib().vio_onion_init(self.h, C.byref(k)))
        return int(k.value)

    def onion_layer(self, Hp, layer):
        """One onion-peel layer: returns (erosion of Hp, layer mask, target
        mask, reconstructed values [|layer|][5] in [0,1])."""
        E = np.ascontiguousarray(Hp, np.uint8).copy()
        bd = np.zeros_like(E)
        S = np.zeros_like(E)
        n = C.c_int64(0)
        nb = int(np.count_nonzero(Hp))
        out = np.zeros((max(nb, 1), 5), np.float32)
        _check("vio_onion_layer", lib().vio_onion_layer(
            self.h, _ptr(E, C.c_uint8), layer, _ptr(bd, C.c_uint8), _ptr(S, C.c_uint8),
            _ptr(out, C.c_float), C.byref(n)))
        return E, bd, S, out[:int(n.value)]

    @property
    def patch_dim(self):
        return 5 * self.params.patch[0] * self.params.patch[1] * self.params.patch[2]

    def pca_moments(self, level, n_max=65536):
        """(S1 [dim], S2 [dim][dim], n): exact moments of the sampled source
        patches."""
        dim = self.patch_dim
        S1 = np.zeros(dim, np.uint64)
        S2 = np.zeros((dim, dim), np.uint64)
        n = C.c_int64(0)
        _check("vio_pca_moments", lib().vio_pca_moments(
            self.h, level, n_max, _ptr(S1, C.c_uint64), _ptr(S2, C.c_uint64), C.byref(n)))
        return S1, S2, int(n.value)

    def pca_basis(self, level, d, n_max=65536):
        """Q [d][dim] int16: the quantised d leading principal directions of
        the level's source patches."""
        from . import pca
        S1, S2, n = self.pca_moments(level, n_max)
        _, B = pca.basis(pca.covariance(S1, S2, n, self.params.lambda_), d)
        return pca.quantize(B, self.params.lambda_)

    def set_reduction(self, level, Q):
        """Searches at this level compare the features of basis Q [d][dim]
        (None: the exact distance again)."""
        if Q is None:
            _check("vio_set_reduction", lib().vio_set_reduction(self.h, level, None, 0))
            return
        q = np.ascontiguousarray(Q, np.int16)
        _check("vio_set_reduction", lib().vio_set_reduction(self.h, level, _ptr(q, C.c_int16),
                                                            q.shape[0]))

    def features(self, level, d):
        W, H, T = self.dims(level)
        out = np.zeros((T, H, W, d), np.int32)
        _check("vio_features", lib().vio_features(self.h, level, _ptr(out, C.c_int32)))
        return out

    def rs_candidate(self, level, p, c0, k, step=0):
        return int(lib().vio_rs_candidate(self.h, level, int(p), int(c0), int(k),
                                          C.c_uint64(int(step))))

    def transition(self, level):
        _check("vio_transition", lib().vio_transition(self.h, level))

    def inpaint(self):
        out = np.zeros((self.T, self.H, self.W, 3), np.uint8)
        _check("vio_inpaint", lib().vio_inpaint(self.h, _ptr(out, C.c_uint8)))
        return out

    def energy(self, level):
        return int(lib().vio_energy(self.h, level))


def num_threads():
    return int(lib().vio_num_threads())


# ---------------------------------------------------------------- realignment

def align_params(**kw) -> AlignParams:
    p = AlignParams()
    _check("vio_align_params_default", lib().vio_align_params_default(C.byref(p)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def align_estimate(video, mask, **kw):
    """theta [T-1][6]: the dominant affine motion of every frame pair."""
    v = np.ascontiguousarray(video, np.uint8)
    m = np.ascontiguousarray(mask, np.uint8)
    T, H, W, _ = v.shape
    th = np.zeros((T - 1, 6), np.float64)
    p = align_params(**kw)
    _check("vio_align_estimate", lib().vio_align_estimate(
        _ptr(v, C.c_uint8), _ptr(m, C.c_uint8), W, H, T, C.byref(p), _ptr(th, C.c_double)))
    return th


def align_compose(theta, T):
    th = np.ascontiguousarray(theta, np.float64)
    M = np.zeros((T, 6), np.float64)
    _check("vio_align_compose", lib().vio_align_compose(_ptr(th, C.c_double), T,
                                                        _ptr(M, C.c_double)))
    return M


def align_warp(video, mask, M):
    v = np.ascontiguousarray(video, np.uint8)
    m = np.ascontiguousarray(mask, np.uint8)
    T, H, W, _ = v.shape
    Mm = np.ascontiguousarray(M, np.float64)
    out = np.zeros_like(v)
    om = np.zeros_like(m)
    _check("vio_align_warp", lib().vio_align_warp(
        _ptr(v, C.c_uint8), _ptr(m, C.c_uint8), W, H, T, _ptr(Mm, C.c_double),
        _ptr(out, C.c_uint8), _ptr(om, C.c_uint8)))
    return out, om


def align_unwarp(aligned, video, mask, M):
    a = np.ascontiguousarray(aligned, np.uint8)
    v = np.ascontiguousarray(video, np.uint8)
    m = np.ascontiguousarray(mask, np.uint8)
    T, H, W, _ = v.shape
    Mm = np.ascontiguousarray(M, np.float64)
    out = np.zeros_like(v)
    _check("vio_align_unwarp", lib().vio_align_unwarp(
        _ptr(a, C.c_uint8), _ptr(v, C.c_uint8), _ptr(m, C.c_uint8), W, H, T,
        _ptr(Mm, C.c_double), _ptr(out, C.c_uint8)))
    return out


# ------------------------------------------------ App. B textured-patch count

def closer_than_constant(ref, vol, patch, mu=128):
    """counts[r]: patches V of the grey volume ``vol`` [T][H][W] with
    SSD(ref[r], V) < SSD(ref[r], Z), Z the constant patch ``mu``; ``ref`` is
    [n][pt][ph][pw] (or [n][N]) and ``patch`` = (pw, ph, pt)."""
    pw, ph, pt = patch
    r = np.ascontiguousarray(ref, np.uint8).reshape(-1, pw * ph * pt)
    v = np.ascontiguousarray(vol, np.uint8)
    T, H, W = v.shape
    out = np.zeros(r.shape[0], np.uint64)
    _check("vio_closer_than_constant", lib().vio_closer_than_constant(
        _ptr(r, C.c_uint8), r.shape[0], _ptr(v, C.c_uint8), W, H, T, pw, ph, pt, mu,
        _ptr(out, C.c_uint64)))
    return out
