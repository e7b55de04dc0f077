"""ctypes wrapper around the C oracle -- TEST INFRASTRUCTURE ONLY.

The oracle (``gakco_oracle.c`` beside this file) is the plain CPU statement of
GaKCo's gapped k-mer kernel (Singh et al. 2017, Algorithm 1 with Eqs. 5-9)
that the GPU library is checked against.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this module.  It imports
nothing from the GPU package.

All arrays are numpy; sequences are passed as one concatenated int8 array of
symbol codes plus an int32 array of lengths.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gakco_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            lib.orc_binomial.argtypes = [ctypes.c_int, ctypes.c_int]
            lib.orc_binomial.restype = i64
            lib.orc_total_gmers.argtypes = [P, i32, i32]
            lib.orc_total_gmers.restype = i64
            lib.orc_gmers.argtypes = [P, P, i32, i32, P, P, i64]
            lib.orc_gmers.restype = i64
            lib.orc_mismatch_profile.argtypes = [P, P, i32, i32, i32, i32, i32, P, P]
            lib.orc_mismatch_profile.restype = ctypes.c_int
            lib.orc_kernel.argtypes = [P, P, i32, i32, i32, i32, i32, P, P, P, P]
            lib.orc_kernel.restype = ctypes.c_int
            lib.orc_mask_groups.argtypes = [P, P, i32, i32, P, i32, P, P, i64, P, P, i64]
            lib.orc_mask_groups.restype = i64
            lib.orc_rows.argtypes = [P, P, i32, P, P, i32, i32, i32, P, f64, i32, P, P, P]
            lib.orc_rows.restype = ctypes.c_int
            lib.orc_svm_dcd.argtypes = [P, P, i32, f64, f64, i32, P, P, P, P]
            lib.orc_svm_dcd.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(seqs, lens):
    seqs = np.ascontiguousarray(seqs, dtype=np.int8)
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    if seqs.size == 0:
        seqs = np.zeros(1, dtype=np.int8)
    return seqs, lens


def host_threads(cap: int = 16) -> int:
    """Threads for full-size oracle runs: the host's cores, at most `cap`."""
    return max(1, min(cap, os.cpu_count() or 1))


def binomial(n: int, r: int) -> int:
    return int(_load().orc_binomial(n, r))


def gmers(seqs, lens, g):
    """The g-mer array L (Section 2.2 step 1): ([T, g] uint8 symbols, [T] sequence ids)."""
    lib = _load()
    seqs, lens = _prep(seqs, lens)
    T = int(lib.orc_total_gmers(_ptr(lens), len(lens), g))
    sym = np.zeros((max(T, 1), g), dtype=np.uint8)
    sid = np.zeros(max(T, 1), dtype=np.int32)
    rc = lib.orc_gmers(_ptr(seqs), _ptr(lens), len(lens), g, _ptr(sym), _ptr(sid), T)
    if rc < 0:
        raise RuntimeError("orc_gmers failed: %d" % rc)
    return sym[:T], sid[:T]


def mismatch_profile(seqs, lens, g, M, threads: int = 1, per_mask: bool = False):
    """(C, N): cumulative and exact mismatch profiles, each [M+1, N, N] int64.

    threads > 1 runs one thread per m (Section 2.2), or with per_mask the
    position sets dealt to `threads` threads (Section S:5.3)."""
    lib = _load()
    seqs, lens = _prep(seqs, lens)
    N = len(lens)
    C = np.zeros((M + 1, N, N), dtype=np.int64)
    Nm = np.zeros((M + 1, N, N), dtype=np.int64)
    rc = lib.orc_mismatch_profile(_ptr(seqs), _ptr(lens), N, g, M, threads, int(per_mask), _ptr(C), _ptr(Nm))
    if rc != 0:
        raise RuntimeError("orc_mismatch_profile failed: %d" % rc)
    return C, Nm


def kernel(seqs, lens, g, k, threads: int = 1, want_c: bool = True, want_nm: bool = True,
           per_mask: bool = False):
    """dict with C [M+1,N,N], Nm [M+1,N,N], K [N,N] int64 and Kn [N,N] float64.

    threads / per_mask as in mismatch_profile."""
    lib = _load()
    seqs, lens = _prep(seqs, lens)
    N = len(lens)
    M = g - k
    C = np.zeros((M + 1, N, N), dtype=np.int64) if want_c else None
    Nm = np.zeros((M + 1, N, N), dtype=np.int64) if want_nm else None
    K = np.zeros((N, N), dtype=np.int64)
    Kn = np.zeros((N, N), dtype=np.float64)
    rc = lib.orc_kernel(_ptr(seqs), _ptr(lens), N, g, k, threads, int(per_mask), _ptr(C), _ptr(Nm), _ptr(K),
                        _ptr(Kn))
    if rc != 0:
        raise RuntimeError("orc_kernel failed: %d" % rc)
    return {"C": C, "Nm": Nm, "K": K, "Kn": Kn}


def mask_groups(seqs, lens, g, removed):
    """Groups of the sorted reduced list for one set of removed positions.

    Returns a list of (rep_index, [(sid, count), ...]) where rep_index is the
    extraction-order index of one g-mer of the group.
    """
    lib = _load()
    seqs, lens = _prep(seqs, lens)
    N = len(lens)
    T = int(lib.orc_total_gmers(_ptr(lens), N, g))
    removed = np.ascontiguousarray(sorted(removed), dtype=np.int32)
    cap = max(T, 1)
    grp_off = np.zeros(cap + 1, dtype=np.int32)
    grp_rep = np.zeros(cap, dtype=np.int32)
    ent_sid = np.zeros(cap, dtype=np.int32)
    ent_cnt = np.zeros(cap, dtype=np.int32)
    ng = lib.orc_mask_groups(_ptr(seqs), _ptr(lens), N, g, _ptr(removed) if len(removed) else None,
                             len(removed), _ptr(grp_off), _ptr(grp_rep), cap,
                             _ptr(ent_sid), _ptr(ent_cnt), cap)
    if ng < 0:
        raise RuntimeError("orc_mask_groups failed: %d" % ng)
    out = []
    for q in range(int(ng)):
        a, b = grp_off[q], grp_off[q + 1]
        out.append((int(grp_rep[q]), list(zip(ent_sid[a:b].tolist(), ent_cnt[a:b].tolist()))))
    return out


def rows(sv_seqs, sv_lens, q_seqs, q_lens, g, k, alpha=None, bias: float = 0.0, threads: int = 1):
    """Kernel rows of queries against a resident set and Eq. 1 decision values.

    Returns dict Krows [n_q, n_sv] float64, Nm [M+1, n_q, n_sv] int64,
    decision [n_q] float64 (None when alpha is None).  threads > 1 deals the
    position sets to that many threads (Section S:5.3).
    """
    lib = _load()
    sv_seqs, sv_lens = _prep(sv_seqs, sv_lens)
    q_seqs, q_lens = _prep(q_seqs, q_lens)
    n_sv, n_q, M = len(sv_lens), len(q_lens), g - k
    Krows = np.zeros((n_q, n_sv), dtype=np.float64)
    Nm = np.zeros((M + 1, n_q, n_sv), dtype=np.int64)
    dec = np.zeros(n_q, dtype=np.float64)
    a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
    rc = lib.orc_rows(_ptr(sv_seqs), _ptr(sv_lens), n_sv, _ptr(q_seqs), _ptr(q_lens), n_q, g, k,
                      _ptr(a), float(bias), int(threads), _ptr(Krows), _ptr(Nm), _ptr(dec))
    if rc != 0:
        raise RuntimeError("orc_rows failed: %d" % rc)
    return {"Krows": Krows, "Nm": Nm, "decision": dec if alpha is not None else None}


def pair_entry(seq_x, seq_y, g, k):
    """One kernel entry computed on the two-sequence dataset {x, y}.

    C_m(x, y), N_m(x, y) and K(x, y) depend only on x and y, so Algorithm 1 on
    the pair gives the entry of the full Gram matrix; the diagonal entries of
    the pair give K(x, x) and K(y, y) for the normalisation.
    Returns (Nm[M+1] int64, K int64, Kn float64).
    """
    sx = np.asarray(seq_x, dtype=np.int8)
    sy = np.asarray(seq_y, dtype=np.int8)
    seqs = np.concatenate([sx, sy])
    lens = np.array([len(sx), len(sy)], dtype=np.int32)
    r = kernel(seqs, lens, g, k, want_c=False)
    return r["Nm"][:, 0, 1].copy(), int(r["K"][0, 1]), float(r["Kn"][0, 1])


def svm_dcd(K, y, C: float = 1.0, eps: float = 1e-8, max_epochs: int = 10000):
    """The SVM of Eq. 1 trained on a normalised kernel K [N,N] with labels y
    (+1/-1) by dual coordinate descent (bias absorbed as K + 1).

    Returns dict alpha [N], dual_coef [N] (alpha_i y_i), bias, epochs."""
    lib = _load()
    K = np.ascontiguousarray(K, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.int8)
    N = len(y)
    alpha = np.zeros(N, dtype=np.float64)
    dual = np.zeros(N, dtype=np.float64)
    b = ctypes.c_double()
    ep = ctypes.c_int32()
    rc = lib.orc_svm_dcd(_ptr(K), _ptr(y), N, float(C), float(eps), int(max_epochs), _ptr(alpha), _ptr(dual),
                         ctypes.byref(b), ctypes.byref(ep))
    if rc != 0:
        raise RuntimeError("orc_svm_dcd failed: %d" % rc)
    return {"alpha": alpha, "dual_coef": dual, "bias": b.value, "epochs": ep.value}
