"""ctypes binding of libdsrg.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels.  PyTorch is used only
for device memory and the current stream when the caller passes device tensors.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsrg.so")

DSRG_OK = 0
DSRG_E_ARG = -1
DSRG_E_NONFINITE = -2
DSRG_E_OOM = -3
DSRG_E_HIP = -4
DSRG_E_UNSUPPORTED = -5
DSRG_E_RDM = -6
DSRG_E_INTRUDER = -7
DSRG_F_DEVICE_PTRS = 1
DSRG_F_PROFILE = 2
DSRG_F_NO_GROUPING = 4
DSRG_F_NO_PLAN_CACHE = 8
DSRG_F_FULL_LADDER = 16
DSRG_PRECISION_FP64 = 0
DSRG_PRECISION_FP32 = 1
DSRG_PRECISION_BF16X3 = 2
MLP_FEATURES = 16
MLP_WEIGHTS_BYTES = 141572

_dp = ctypes.POINTER(ctypes.c_double)


class Problem(ctypes.Structure):
    _fields_ = [("n_core", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("n_virtual", ctypes.c_int32), ("n_aux", ctypes.c_int32),
                ("eps", ctypes.c_void_p), ("B", ctypes.c_void_p), ("gamma1", ctypes.c_void_p),
                ("gamma2", ctypes.c_void_p), ("gamma3", ctypes.c_void_p), ("s", ctypes.c_double),
                ("f_offdiag", ctypes.c_void_p), ("e0", ctypes.c_double)]


class TileRule(ctypes.Structure):
    _fields_ = [("np_min", ctypes.c_int32), ("np_max", ctypes.c_int32),
                ("big_tile_min", ctypes.c_int32), ("virt_batch", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("workspace_cap", ctypes.c_int64), ("stream", ctypes.c_void_p),
                ("virt_batch", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("e2", ctypes.c_double), ("e3", ctypes.c_double), ("e3_a", ctypes.c_double),
                ("e3_b", ctypes.c_double), ("t_seconds", ctypes.c_double * 8),
                ("gett_flops", ctypes.c_double), ("ladder_flops", ctypes.c_double),
                ("ladder_seconds", ctypes.c_double), ("ladder_batch", ctypes.c_int32),
                ("n_launch", ctypes.c_int32), ("role_seconds", ctypes.c_double * 4),
                ("role_flops", ctypes.c_double * 4), ("role_launches", ctypes.c_int32 * 4),
                ("plan", ctypes.c_int32), ("grouped_uses", ctypes.c_int32),
                ("role_bytes", ctypes.c_double * 4), ("e_total", ctypes.c_double),
                ("alg_flops", ctypes.c_double), ("precision_used", ctypes.c_int32),
                ("virt_batch_used", ctypes.c_int32), ("kernel_seconds", ctypes.c_double * 8),
                ("kernel_flops", ctypes.c_double * 8), ("kernel_launches", ctypes.c_int32 * 8)]


class Intermediates(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("t1", "t2", "w1", "w2", "z1", "z2", "u1", "u2")]


class RelaxedResult(ctypes.Structure):
    _fields_ = [("e_relaxed", ctypes.c_double), ("e_unrelaxed", ctypes.c_double),
                ("cas_const", ctypes.c_double), ("residual", ctypes.c_double),
                ("n_det", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RelaxedOutputs(ctypes.Structure):
    _fields_ = [("ci", ctypes.c_void_p), ("hbar1", ctypes.c_void_p), ("hbar2", ctypes.c_void_p),
                ("cas_c", ctypes.c_void_p)]


class DsrgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("dsrg error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libdsrg.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdsrg.so is not built; run paper_1701_02011_amd/_build.py "
                              "or __graft_entry__.build()")
        # One HIP runtime per process: PyTorch-ROCm ships its own libamdhip64.so.7.  Loading
        # torch first makes libdsrg bind to that copy (same SONAME), so device pointers and
        # streams from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for fn in ("dsrg_pt2_energy", "dsrg_pt3_energy"):
            getattr(lib, fn).argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                         ctypes.POINTER(Result)]
            getattr(lib, fn).restype = ctypes.c_int
        lib.dsrg_pt3_energy_ex.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                           ctypes.POINTER(Result), ctypes.POINTER(Intermediates)]
        lib.dsrg_pt3_energy_ex.restype = ctypes.c_int
        lib.dsrg_release_cache.restype = ctypes.c_int
        lib.dsrg_pt3_pair_energies.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                               ctypes.POINTER(Result), _dp, _dp]
        lib.dsrg_pt3_pair_energies.restype = ctypes.c_int
        lib.dsrg_pt3_energy_batch.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32,
                                              ctypes.POINTER(Options), ctypes.POINTER(Result),
                                              ctypes.POINTER(ctypes.c_int32)]
        lib.dsrg_pt3_energy_batch.restype = ctypes.c_int
        lib.dsrg_last_error.restype = ctypes.c_char_p
        lib.dsrg_version.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        lib.dsrg_test_gett.argtypes = [ctypes.c_int, ip, lp, lp, ctypes.c_int, ip, lp, lp,
                                       ctypes.c_int, ip, lp, lp, _dp, ctypes.c_longlong, _dp,
                                       ctypes.c_longlong, _dp, ctypes.c_longlong, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int]
        lib.dsrg_test_gett.restype = ctypes.c_int
        fp = ctypes.POINTER(ctypes.c_float)
        lib.dsrg_pair_features.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), fp, _dp]
        lib.dsrg_pair_features.restype = ctypes.c_int
        lib.dsrg_mlp_train.argtypes = [fp, _dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p]
        lib.dsrg_mlp_train.restype = ctypes.c_int
        lib.dsrg_mlp_predict.argtypes = [ctypes.c_void_p, fp, ctypes.c_int64, _dp]
        lib.dsrg_mlp_predict.restype = ctypes.c_int
        lib.dsrg_pt3_energy_surrogate.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                                  ctypes.c_void_p, ctypes.c_double,
                                                  ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_int32)]
        lib.dsrg_pt3_energy_surrogate.restype = ctypes.c_int
        lib.dsrg_test_mlp_grad.argtypes = [ctypes.c_void_p, fp, _dp, ctypes.c_int64, _dp, fp]
        lib.dsrg_test_mlp_grad.restype = ctypes.c_int
        lib.dsrg_pt3_energy_noalloc.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                                ctypes.POINTER(Result)]
        lib.dsrg_pt3_energy_noalloc.restype = ctypes.c_int
        lib.dsrg_active_rdms.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]
        lib.dsrg_active_rdms.restype = ctypes.c_int
        lib.dsrg_pt3_energy_relaxed.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_void_p, ctypes.POINTER(Options),
                                                ctypes.POINTER(Result), ctypes.POINTER(RelaxedResult),
                                                ctypes.POINTER(RelaxedOutputs)]
        lib.dsrg_pt3_energy_relaxed.restype = ctypes.c_int
        lib.dsrg_dyall_aavv.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_void_p,
                                        ctypes.c_void_p]
        lib.dsrg_dyall_aavv.restype = ctypes.c_int
        lib.dsrg_set_tile_rules.argtypes = [ctypes.POINTER(TileRule), ctypes.c_int32]
        lib.dsrg_set_tile_rules.restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != DSRG_OK:
        raise DsrgError(rc, load().dsrg_last_error().decode())


def _host(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data


_ARRAYS = ("eps", "B", "gamma1", "gamma2", "gamma3", "f_offdiag")


def _problem_struct(p, keep):
    """dsrg_problem from a synth.Problem (host arrays) or a dict of torch device tensors."""
    if isinstance(p, dict):
        fl = DSRG_F_DEVICE_PTRS
        get = lambda k: None if p.get(k) is None else p[k].data_ptr()
        for k in _ARRAYS:
            if p.get(k) is not None:
                keep.append(p[k])
        st = Problem(int(p["n_core"]), int(p["n_active"]), int(p["n_virtual"]), int(p["n_aux"]),
                     get("eps"), get("B"), get("gamma1"), get("gamma2"), get("gamma3"),
                     float(p["s"]), get("f_offdiag"), float(p.get("e0", 0.0)))
        return st, fl
    ptrs = {}
    for k in _ARRAYS:
        arr, ptr = _host(getattr(p, k, None))
        keep.append(arr)
        ptrs[k] = ptr
    st = Problem(p.n_core, p.n_active, p.n_virtual, p.n_aux, ptrs["eps"], ptrs["B"],
                 ptrs["gamma1"], ptrs["gamma2"], ptrs["gamma3"], float(p.s), ptrs["f_offdiag"],
                 float(getattr(p, "e0", 0.0)))
    return st, 0


def _options(flags, stream=None, workspace_cap=0, precision=DSRG_PRECISION_FP64, virt_batch=0):
    return Options(flags, int(precision), int(workspace_cap), stream, int(virt_batch))


def to_device(p, device="cuda:0"):
    """Copy a synth.Problem's arrays into torch device tensors (marshalling helper)."""
    import torch
    d = dict(n_core=p.n_core, n_active=p.n_active, n_virtual=p.n_virtual, n_aux=p.n_aux, s=p.s,
             e0=float(getattr(p, "e0", 0.0)))
    for k in _ARRAYS:
        a = getattr(p, k, None)
        d[k] = None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return d


def _result_dict(r: Result):
    return dict(e2=r.e2, e3=r.e3, e3_a=r.e3_a, e3_b=r.e3_b, t_seconds=list(r.t_seconds),
                gett_flops=r.gett_flops, ladder_flops=r.ladder_flops,
                ladder_seconds=r.ladder_seconds, ladder_batch=r.ladder_batch,
                n_launch=r.n_launch, role_seconds=list(r.role_seconds),
                role_flops=list(r.role_flops), role_launches=list(r.role_launches), plan=r.plan,
                grouped_uses=r.grouped_uses, role_bytes=list(r.role_bytes), e_total=r.e_total,
                alg_flops=r.alg_flops, precision_used=r.precision_used,
                virt_batch_used=r.virt_batch_used, kernel_seconds=list(r.kernel_seconds),
                kernel_flops=list(r.kernel_flops), kernel_launches=list(r.kernel_launches))


def _stream_of(p, stream):
    if stream is not None:
        return stream
    if isinstance(p, dict):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


def _flags(fl, profile=False, grouping=True, cache=True, unique_ladder=True):
    if not unique_ladder:
        fl |= DSRG_F_FULL_LADDER
    if profile:
        fl |= DSRG_F_PROFILE
    if not grouping:
        fl |= DSRG_F_NO_GROUPING
    if not cache:
        fl |= DSRG_F_NO_PLAN_CACHE
    return fl


def release_cache():
    """Free the library's cached plans (device buffers and graphs)."""
    _check(load().dsrg_release_cache())


def dsrg_pt2_energy(p, stream=None, workspace_cap=0, grouping=True, cache=True, precision=0,
                    virt_batch=0):
    keep = []
    st, fl = _problem_struct(p, keep)
    fl = _flags(fl, grouping=grouping, cache=cache)
    r = Result()
    _check(load().dsrg_pt2_energy(ctypes.byref(st), ctypes.byref(
        _options(fl, _stream_of(p, stream), workspace_cap, precision, virt_batch)), ctypes.byref(r)))
    return _result_dict(r)


def dsrg_pt3_energy(p, stream=None, workspace_cap=0, profile=False, grouping=True, cache=True,
                    precision=0, unique_ladder=True, virt_batch=0):
    keep = []
    st, fl = _problem_struct(p, keep)
    fl = _flags(fl, profile, grouping, cache, unique_ladder)
    r = Result()
    _check(load().dsrg_pt3_energy(ctypes.byref(st), ctypes.byref(
        _options(fl, _stream_of(p, stream), workspace_cap, precision, virt_batch)), ctypes.byref(r)))
    return _result_dict(r)


def dsrg_pt3_energy_batch(problems, stream=None, workspace_cap=0, precision=0, grouping=True,
                          cache=True):
    """E(2), E(3) of several problems in one call: (list of result dicts or None, codes).
    All problems must be host problems or all device dicts."""
    keep = []
    structs, flags = [], set()
    for p in problems:
        st, fl = _problem_struct(p, keep)
        structs.append(st)
        flags.add(fl)
    if len(flags) > 1:
        raise ValueError("mix of host and device problems")
    n = len(structs)
    arr = (Problem * n)(*structs)
    res = (Result * n)()
    status = (ctypes.c_int32 * n)()
    fl = _flags(flags.pop() if flags else 0, grouping=grouping, cache=cache)
    st0 = _stream_of(problems[0], stream) if problems else None
    rc = load().dsrg_pt3_energy_batch(arr, n, ctypes.byref(_options(fl, st0, workspace_cap, precision)),
                                      res, status)
    codes = list(status)
    if rc != DSRG_OK and not any(c == DSRG_OK for c in codes):
        _check(rc)
    return [(_result_dict(res[k]) if codes[k] == DSRG_OK else None) for k in range(n)], codes


def dsrg_pt3_pair_energies(p, stream=None, workspace_cap=0, precision=0, grouping=True):
    """E(2), E(3) and the core-pair decomposition of E(3): the result dict gains
    'pairs' {(i, j): e_ij} for core orbitals i <= j and 'rest'."""
    keep = []
    st, fl = _problem_struct(p, keep)
    nC = int(st.n_core)
    buf = np.zeros(max(1, nC * (nC + 1) // 2))
    rest = np.zeros(1)
    r = Result()
    _check(load().dsrg_pt3_pair_energies(ctypes.byref(st), ctypes.byref(
        _options(_flags(fl, grouping=grouping), _stream_of(p, stream), workspace_cap, precision)),
        ctypes.byref(r), buf.ctypes.data_as(_dp), rest.ctypes.data_as(_dp)))
    out = _result_dict(r)
    keys = [(i, j) for i in range(nC) for j in range(i, nC)]
    out["pairs"] = {k: float(buf[n]) for n, k in enumerate(keys)}
    out["rest"] = float(rest[0])
    return out


INTERMEDIATES = ("t1", "t2", "w1", "w2", "z1", "z2", "u1", "u2")


def dsrg_pt3_energy_ex(p, stream=None, workspace_cap=0, grouping=True, precision=0,
                       keys=INTERMEDIATES, unique_ladder=True, virt_batch=0):
    """E(2), E(3) and the requested intermediates as numpy arrays (spin blocks, excitation
    order)."""
    keep = []
    st, fl = _problem_struct(p, keep)
    fl = _flags(fl, grouping=grouping, unique_ladder=unique_ladder)
    nC, nA, nV = st.n_core, st.n_active, st.n_virtual
    nH, nP = nC + nA, nA + nV
    bufs = {}
    for k in keys:
        bufs[k] = np.zeros((2, nP, nH)) if k.endswith("1") else np.zeros((3, nP, nP, nH, nH))
    inter = Intermediates(**{k: v.ctypes.data for k, v in bufs.items()})
    r = Result()
    _check(load().dsrg_pt3_energy_ex(ctypes.byref(st), ctypes.byref(
        _options(fl, _stream_of(p, stream), workspace_cap, precision, virt_batch)), ctypes.byref(r),
        ctypes.byref(inter)))
    out = _result_dict(r)
    out.update(bufs)
    return out


def test_gett(A, B, C, m, n, k, alpha=1.0, beta=0, precision=0):
    """Run the contraction kernel once.  m, n, k: lists of (extent, strideA-or-B, strideC)
    triples: m -> (extent, A stride, C stride), n -> (extent, B stride, C stride),
    k -> (extent, A stride, B stride)."""
    A = np.ascontiguousarray(A, dtype=np.float64).ravel()
    B = np.ascontiguousarray(B, dtype=np.float64).ravel()
    C = np.ascontiguousarray(C, dtype=np.float64).ravel().copy()
    I = lambda v: (ctypes.c_int * max(1, len(v)))(*v)
    L = lambda v: (ctypes.c_longlong * max(1, len(v)))(*v)
    rc = load().dsrg_test_gett(len(m), I([x[0] for x in m]), L([x[1] for x in m]), L([x[2] for x in m]),
                               len(n), I([x[0] for x in n]), L([x[1] for x in n]), L([x[2] for x in n]),
                               len(k), I([x[0] for x in k]), L([x[1] for x in k]), L([x[2] for x in k]),
                               A.ctypes.data_as(_dp), A.size, B.ctypes.data_as(_dp), B.size,
                               C.ctypes.data_as(_dp), C.size, float(alpha), int(beta),
                               int(precision))
    _check(rc)
    return C


# ---------------------------------------------------------------------------
# the pair-energy network
# ---------------------------------------------------------------------------
def _f32(a, cols=None):
    arr = np.ascontiguousarray(a, dtype=np.float32)
    if cols is not None:
        arr = arr.reshape(-1, cols)
    return arr


def dsrg_pair_features(p, stream=None):
    """(features [nC(nC+1)/2][16] float32, E2_ij proxies [nC(nC+1)/2]) of the core pairs."""
    keep = []
    st, fl = _problem_struct(p, keep)
    nC = int(st.n_core)
    np_ = max(1, nC * (nC + 1) // 2)
    X = np.zeros((np_, MLP_FEATURES), dtype=np.float32)
    e2 = np.zeros(np_)
    _check(load().dsrg_pair_features(ctypes.byref(st), ctypes.byref(_options(fl, _stream_of(p, stream))),
                                     X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), e2.ctypes.data_as(_dp)))
    n = nC * (nC + 1) // 2
    return X[:n], e2[:n]


def dsrg_mlp_train(X, y, epochs=2000, seed=1):
    """Train the network on the GPU; returns the weights blob (bytes)."""
    X = _f32(X, MLP_FEATURES)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = ctypes.create_string_buffer(MLP_WEIGHTS_BYTES)
    _check(load().dsrg_mlp_train(X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), y.ctypes.data_as(_dp),
                                 len(y), int(epochs), int(seed), out))
    return out.raw


def dsrg_mlp_predict(weights, X):
    X = _f32(X, MLP_FEATURES)
    y = np.zeros(len(X))
    buf = ctypes.create_string_buffer(bytes(weights), MLP_WEIGHTS_BYTES)
    _check(load().dsrg_mlp_predict(buf, X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), len(X),
                                   y.ctypes.data_as(_dp)))
    return y


def test_mlp_grad(weights, X, y):
    """(loss, gradient) of the network at the given weights, from the training kernels."""
    X = _f32(X, MLP_FEATURES)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.zeros(MLP_WEIGHTS_BYTES // 4 - 64, dtype=np.float32)
    loss = ctypes.c_double(0.0)
    buf = ctypes.create_string_buffer(bytes(weights), MLP_WEIGHTS_BYTES)
    _check(load().dsrg_test_mlp_grad(buf, X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     y.ctypes.data_as(_dp), len(y), ctypes.byref(loss),
                                     g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return loss.value, g


def dsrg_pt3_energy_surrogate(p, weights, rel_threshold=1.0, stream=None, workspace_cap=0, precision=0):
    """E(2) and E(3) with the core-pair parts of E(3) from the network (exact fallback per
    rel_threshold); the result dict gains 'n_exact_pairs'."""
    keep = []
    st, fl = _problem_struct(p, keep)
    r = Result()
    nex = ctypes.c_int32(0)
    buf = ctypes.create_string_buffer(bytes(weights), MLP_WEIGHTS_BYTES)
    _check(load().dsrg_pt3_energy_surrogate(ctypes.byref(st), ctypes.byref(
        _options(fl, _stream_of(p, stream), workspace_cap, precision)), buf, float(rel_threshold),
        ctypes.byref(r), ctypes.byref(nex)))
    out = _result_dict(r)
    out["n_exact_pairs"] = nex.value
    return out


def dsrg_active_rdms(ci, n_active, n_alpha, n_beta, with_gamma3=True):
    """gamma1 [2][nA]^2, gamma2 [3][nA]^4, gamma3 [4][nA]^6 (or None) of a CAS vector, on the
    GPU (host arrays in and out)."""
    c = np.ascontiguousarray(ci, dtype=np.float64)
    nA = int(n_active)
    g1 = np.zeros((2,) + (nA,) * 2)
    g2 = np.zeros((3,) + (nA,) * 4)
    g3 = np.zeros((4,) + (nA,) * 6) if with_gamma3 else None
    _check(load().dsrg_active_rdms(c.ctypes.data, nA, int(n_alpha), int(n_beta),
                                   ctypes.byref(_options(0)), g1.ctypes.data, g2.ctypes.data,
                                   None if g3 is None else g3.ctypes.data))
    return g1, g2, g3


def dsrg_pt3_energy_relaxed(p, n_alpha=None, n_beta=None, ci_guess="reference", stream=None,
                            workspace_cap=0, precision=0, outputs=True):
    """E(2), E(3) and the one-step relaxed energy.  n_alpha/n_beta default to the problem's;
    ci_guess "reference" passes the problem's CI vector (None: no guess).  With outputs the
    dict gains 'ci', 'hbar1', 'hbar2', 'cas_c' (numpy arrays)."""
    keep = []
    st, fl = _problem_struct(p, keep)
    nA = st.n_active
    na = int(p.n_alpha if n_alpha is None else n_alpha)
    nb = int(p.n_beta if n_beta is None else n_beta)
    guess = None
    if isinstance(ci_guess, str):
        if getattr(p, "ci", None) is not None:
            guess = np.ascontiguousarray(np.asarray(p.ci), dtype=np.float64)
    elif ci_guess is not None:
        guess = np.ascontiguousarray(ci_guess, dtype=np.float64)
    ndet = math.comb(nA, na) * math.comb(nA, nb) if 0 <= na <= nA and 0 <= nb <= nA else 0
    bufs = {}
    if outputs:
        bufs = dict(ci=np.zeros(max(ndet, 1)), hbar1=np.zeros((2, nA, nA)), hbar2=np.zeros((3,) + (nA,) * 4),
                    cas_c=np.zeros((2, nA, nA)))
    o = RelaxedOutputs(**{k: v.ctypes.data for k, v in bufs.items()})
    r = Result()
    x = RelaxedResult()
    _check(load().dsrg_pt3_energy_relaxed(ctypes.byref(st), na, nb,
                                          None if guess is None else guess.ctypes.data,
                                          ctypes.byref(_options(fl, _stream_of(p, stream), workspace_cap,
                                                                precision)),
                                          ctypes.byref(r), ctypes.byref(x), ctypes.byref(o)))
    out = _result_dict(r)
    out.update(e_relaxed=x.e_relaxed, e_unrelaxed=x.e_unrelaxed, cas_const=x.cas_const,
               residual=x.residual, n_det=x.n_det, iterations=x.iterations, converged=bool(x.converged))
    if outputs:
        bufs["ci"] = bufs["ci"][:ndet]
        out.update(bufs)
    return out


def dsrg_dyall_aavv(p, stream=None):
    """Active-to-virtual doubles under Dyall's H(0) (host problem in, host arrays out):
    returns (t [3][nV][nV][nA][nA] with blocks aa, ab, bb, smallest |shifted denominator|)."""
    keep = []
    st, fl = _problem_struct(p, keep)
    nA, nV = st.n_active, st.n_virtual
    t = np.zeros((3, nV, nV, nA, nA))
    dmin = ctypes.c_double(0.0)
    _check(load().dsrg_dyall_aavv(ctypes.byref(st), ctypes.byref(_options(fl, stream)), t.ctypes.data,
                                  ctypes.addressof(dmin)))
    return t, dmin.value


TILE_RULES_PATH = os.path.join(HERE, "tile_rules.json")


def set_tile_rules(rules):
    """Install a rule table (list of dicts with np_min, np_max, big_tile_min, virt_batch);
    an empty list restores the built-in choices."""
    arr = (TileRule * max(1, len(rules)))()
    for k, r in enumerate(rules):
        arr[k] = TileRule(int(r["np_min"]), int(r["np_max"]), int(r.get("big_tile_min", 0)),
                          int(r.get("virt_batch", 0)))
    _check(load().dsrg_set_tile_rules(arr, len(rules)))


def load_tile_rules(path=None):
    """Install the autotuner's stored rule table (tile_rules.json beside this module);
    returns the rules, or None when there is no such file."""
    import json
    path = path or TILE_RULES_PATH
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rules = json.load(f)["rules"]
    set_tile_rules(rules)
    return rules
