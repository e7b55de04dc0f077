"""Python binding of libgakco.so (the gfx950 gapped k-mer kernel library).

Argument marshalling only: every step of the computation runs in the HIP
library; torch supplies device memory and the current stream.  Importing this
module does not touch the GPU; loading the library fails loudly when it has
not been built.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgakco.so")

OK, EINVAL, ERANGE, EUNSUPPORTED, EBUDGET, EHIP, ECANCELLED, EAGAIN = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {EINVAL: "EINVAL", ERANGE: "ERANGE", EUNSUPPORTED: "EUNSUPPORTED", EBUDGET: "EBUDGET",
          EHIP: "EHIP", ECANCELLED: "ECANCELLED", EAGAIN: "EAGAIN"}

_lib = None
_lock = threading.Lock()


class GakcoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_NAMES.get(status, "?"), status, msg))
        self.status = status


class Job(ctypes.Structure):
    _fields_ = [("seqs", ctypes.c_void_p), ("lens", ctypes.c_void_p), ("N", ctypes.c_int32),
                ("sigma", ctypes.c_int32), ("g", ctypes.c_int32), ("k", ctypes.c_int32),
                ("K_out", ctypes.c_void_p), ("Nm_out", ctypes.c_void_p), ("status_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("decision", ctypes.c_double),
                ("K_row", ctypes.c_void_p), ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("batch_size", ctypes.c_int32)]


def lib():
    """Load libgakco.so (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libgakco.so is not built (run __graft_entry__.build())")
            L = ctypes.CDLL(LIB_PATH)
            P, i32, i64, sz, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
            sig = {
                "gakco_last_error": ([], ctypes.c_char_p),
                "gakco_version": ([], ctypes.c_char_p),
                "gakco_ctx_create": ([ctypes.c_int, sz, ctypes.c_char_p, P], i32),
                "gakco_ctx_destroy": ([P], None),
                "gakco_ctx_set_param": ([P, ctypes.c_char_p, i64], i32),
                "gakco_count_gmers": ([P, i32, i32, P], i32),
                "gakco_gram": ([P, P, P, i32, i32, i32, i32, P, P, P, P], i32),
                "gakco_extract": ([P, P, P, i32, i32, i32, P, P, P], i32),
                "gakco_mask_groups": ([P, P, P, i32, i32, i32, P, i32, P, P, P, P, i64, P, P], i32),
                "gakco_gram_batch": ([P, P, i32, P], i32),
                "gakco_batch_plan_create": ([P, P, i32, P, P], i32),
                "gakco_batch_run": ([P, P], i32),
                "gakco_batch_plan_destroy": ([P], None),
                "gakco_resident_create": ([P, P, P, i32, i32, i32, i32, P, f64, P], i32),
                "gakco_resident_destroy": ([P], None),
                "gakco_resident_info": ([P, P, P, P, P, P], i32),
                "gakco_rows": ([P, P, P, P, i32, P, P, P, P], i32),
                "gakco_server_create": ([P, i32, i32, i32, sz, P], i32),
                "gakco_server_submit": ([P, P, i32, ctypes.c_uint64], i32),
                "gakco_server_cancel": ([P, ctypes.c_uint64], i32),
                "gakco_server_poll": ([P, P, i32, P, i32], i32),
                "gakco_server_set_param": ([P, ctypes.c_char_p, i64], i32),
                "gakco_server_destroy": ([P], i32),
                "gakco_ctx_stat": ([P, ctypes.c_char_p, P], i32),
                "gakco_autotune": ([P, P, i32, i32, P, ctypes.c_char_p, sz], i32),
                "gakco_profile_phases": ([], i32),
                "gakco_profile_get": ([P, i32, P, P, P], i32),
                "gakco_profile_reset": ([P], None),
                "gakco_probe_lds_atomics": ([P, i32, P], i32),
                "gakco_svm_train": ([P, P, P, i32, f64, f64, i32, P, P, P, P, P], i32),
                "gakco_incr_create": ([P, i32, i32, i32, P], i32),
                "gakco_incr_append": ([P, P, P, i32, P, P, P], i32),
                "gakco_incr_info": ([P, P, P], i32),
                "gakco_incr_destroy": ([P], None),
                "gakco_gram_noalloc": ([P, P, i32, i32, i32, i32, P, P, P, P], i32),
            }
            missing = [name for name in sig if getattr(L, name, None) is None]
            if missing:
                raise RuntimeError("libgakco.so lacks %s: rebuild it (__graft_entry__.build())" % ", ".join(missing))
            for name, (args, res) in sig.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = res
            _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise GakcoError(status, lib().gakco_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_inputs(seqs, lens, device):
    seqs = torch.as_tensor(seqs).to(device=device, dtype=torch.int8).contiguous()
    lens = torch.as_tensor(lens).to(device=device, dtype=torch.int32).contiguous()
    if seqs.numel() == 0:
        seqs = torch.zeros(1, dtype=torch.int8, device=device)
    return seqs, lens


class Context:
    """A device, a scratch arena bounded by `hbm_budget` bytes, tuning knobs."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, tune: dict | None = None):
        import json
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        js = json.dumps(tune).encode() if tune else None
        _check(lib().gakco_ctx_create(device, hbm_budget, js, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().gakco_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_param(self, name: str, value: int):
        _check(lib().gakco_ctx_set_param(self._h, name.encode(), int(value)))

    def profile(self) -> dict:
        """{phase: (total_ms, launches)} from the event profiler."""
        out = {}
        for i in range(lib().gakco_profile_phases()):
            nm, ms, n = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_int64()
            _check(lib().gakco_profile_get(self._h, i, ctypes.byref(nm), ctypes.byref(ms), ctypes.byref(n)))
            out[nm.value.decode()] = (ms.value, n.value)
        return out

    def profile_reset(self):
        lib().gakco_profile_reset(self._h)

    def probe_lds_atomics(self, row_words: int = 4096) -> float:
        """Random-address LDS atomic adds per second (the row accumulation's
        reference rate) over a row of row_words counters."""
        v = ctypes.c_double()
        _check(lib().gakco_probe_lds_atomics(self._h, row_words, ctypes.byref(v)))
        return v.value

    def stat(self, name: str) -> int:
        v = ctypes.c_int64()
        _check(lib().gakco_ctx_stat(self._h, name.encode(), ctypes.byref(v)))
        return v.value

    def svm_train(self, K, y, C: float = 1.0, eps: float = 1e-3, max_epochs: int = 10000):
        """The SVM of Eq. 1 on a device kernel K [N,N] (f64) with labels y
        (+1/-1): dict alpha, dual_coef (device f64 [N]), bias, epochs."""
        N = int(K.shape[0])
        K = K.contiguous()
        y = torch.as_tensor(y).to(device=self.device, dtype=torch.int8).contiguous()
        alpha = torch.empty(N, dtype=torch.float64, device=self.device)
        dual = torch.empty(N, dtype=torch.float64, device=self.device)
        b, ep = ctypes.c_double(), ctypes.c_int32()
        _check(lib().gakco_svm_train(self._h, _ptr(K), _ptr(y), N, float(C), float(eps), int(max_epochs),
                                     _ptr(alpha), _ptr(dual), ctypes.byref(b), ctypes.byref(ep), _stream(self.device)))
        return {"alpha": alpha, "dual_coef": dual, "bias": b.value, "epochs": ep.value}

    # ------------------------------------------------------------- batches --
    def _jobs(self, jobs):
        """jobs: list of dicts with seqs, lens (device tensors), sigma, g, k and
        optional K / Nm output tensors; missing outputs are allocated."""
        arr = (Job * len(jobs))()
        status = (ctypes.c_int32 * len(jobs))()
        keep = []
        for i, j in enumerate(jobs):
            seqs, lens = _dev_inputs(j["seqs"], j["lens"], self.device)
            N, M = int(lens.numel()), j["g"] - j["k"]
            if "K" not in j:
                j["K"] = torch.empty((N, N), dtype=torch.float64, device=self.device)
            if "Nm" not in j:
                j["Nm"] = torch.empty((M + 1, N, N), dtype=torch.int64, device=self.device)
            j["_seqs"], j["_lens"] = seqs, lens
            keep += [seqs, lens]
            arr[i] = Job(seqs.data_ptr(), lens.data_ptr(), N, j["sigma"], j["g"], j["k"],
                         j["K"].data_ptr() if j["K"] is not None else None,
                         j["Nm"].data_ptr() if j["Nm"] is not None else None,
                         ctypes.addressof(status) + 4 * i)
        return arr, status, keep

    def gram_batch(self, jobs):
        """Run every job in shared launches; returns the per-job statuses."""
        arr, status, _keep = self._jobs(jobs)
        rc = lib().gakco_gram_batch(self._h, arr, len(jobs), _stream(self.device))
        if rc != OK and rc != ERANGE:
            _check(rc)
        return list(status)

    def batch_plan(self, jobs):
        return BatchPlan(self, jobs)

    def autotune(self, jobs, reps: int = 2) -> str:
        arr, _status, _keep = self._jobs(jobs)
        buf = ctypes.create_string_buffer(4096)
        _check(lib().gakco_autotune(self._h, arr, len(jobs), reps, _stream(self.device), buf, 4096))
        return buf.value.decode()


    # ---------------------------------------------------------------- Gram --
    def gram(self, seqs, lens, sigma: int, g: int, k: int, want_K: bool = True, want_Nm: bool = True,
             want_Cm: bool = False, out: dict | None = None):
        """Normalised kernel K [N,N] f64, N_m [M+1,N,N] i64, C_m [M+1,N,N] i64 (as requested)."""
        seqs, lens = _dev_inputs(seqs, lens, self.device)
        N, M = int(lens.numel()), g - k
        out = dict(out or {})
        if want_K and "K" not in out:
            out["K"] = torch.empty((N, N), dtype=torch.float64, device=self.device)
        if want_Nm and "Nm" not in out:
            out["Nm"] = torch.empty((M + 1, N, N), dtype=torch.int64, device=self.device)
        if want_Cm and "Cm" not in out:
            out["Cm"] = torch.empty((M + 1, N, N), dtype=torch.int64, device=self.device)
        _check(lib().gakco_gram(self._h, _ptr(seqs), _ptr(lens), N, sigma, g, k, _ptr(out.get("K")),
                                _ptr(out.get("Nm")), _ptr(out.get("Cm")), _stream(self.device)))
        return out

    def gram_into(self, seqs, lens, N, sigma, g, k, K=None, Nm=None, Cm=None):
        """Gram on device tensors already in place (no allocation here)."""
        _check(lib().gakco_gram(self._h, _ptr(seqs), _ptr(lens), N, sigma, g, k, _ptr(K), _ptr(Nm), _ptr(Cm),
                                _stream(self.device)))

    def extract(self, seqs, lens, sigma: int, g: int):
        seqs, lens = _dev_inputs(seqs, lens, self.device)
        lh = lens.cpu().numpy()
        T = ctypes.c_int64()
        _check(lib().gakco_count_gmers(lh.ctypes.data_as(ctypes.c_void_p), len(lh), g, ctypes.byref(T)))
        keys = torch.empty(max(T.value, 1), dtype=torch.int64, device=self.device)
        sid = torch.empty(max(T.value, 1), dtype=torch.int32, device=self.device)
        _check(lib().gakco_extract(self._h, _ptr(seqs), _ptr(lens), len(lh), sigma, g, _ptr(keys), _ptr(sid),
                                   _stream(self.device)))
        return keys[:T.value], sid[:T.value]

    def mask_groups(self, seqs, lens, sigma: int, g: int, removed):
        """Groups of one position set: list of (rep_index, [(sid, count), ...])."""
        import numpy as np
        seqs, lens = _dev_inputs(seqs, lens, self.device)
        lh = lens.cpu().numpy()
        T = ctypes.c_int64()
        _check(lib().gakco_count_gmers(lh.ctypes.data_as(ctypes.c_void_p), len(lh), g, ctypes.byref(T)))
        cap = max(T.value, 1)
        rem = np.ascontiguousarray(sorted(removed), dtype=np.int32)
        grp_off = np.zeros(cap + 1, dtype=np.int32)
        grp_rep = np.zeros(cap, dtype=np.int32)
        ent_sid = np.zeros(cap, dtype=np.int32)
        ent_cnt = np.zeros(cap, dtype=np.int32)
        ng = ctypes.c_int64()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().gakco_mask_groups(self._h, _ptr(seqs), _ptr(lens), len(lh), sigma, g,
                                       vp(rem) if len(rem) else None, len(rem), vp(grp_off), vp(grp_rep),
                                       vp(ent_sid), vp(ent_cnt), cap, ctypes.byref(ng), _stream(self.device)))
        out = []
        for q in range(ng.value):
            a, b = grp_off[q], grp_off[q + 1]
            out.append((int(grp_rep[q]), list(zip(ent_sid[a:b].tolist(), ent_cnt[a:b].tolist()))))
        return out


class BatchPlan:
    """A batch whose launch sequence is captured once into a hipGraph."""

    def __init__(self, ctx: Context, jobs):
        self.ctx = ctx
        self.jobs = jobs
        self._arr, self._status, self._keep = ctx._jobs(jobs)
        h = ctypes.c_void_p()
        _check(lib().gakco_batch_plan_create(ctx._h, self._arr, len(jobs), _stream(ctx.device), ctypes.byref(h)))
        self._h = h

    def run(self):
        rc = lib().gakco_batch_run(self._h, _stream(self.ctx.device))
        if rc != OK and rc != ERANGE:
            _check(rc)
        return list(self._status)

    def close(self):
        if getattr(self, "_h", None):
            lib().gakco_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Resident:
    """A resident sequence set (e.g. support vectors) kept as device tables."""

    def __init__(self, ctx: Context, seqs, lens, sigma: int, g: int, k: int, alpha=None, bias: float = 0.0):
        import numpy as np
        self.ctx = ctx
        seqs, lens = _dev_inputs(seqs, lens, ctx.device)
        self.n_sv, self.sigma, self.g, self.k = int(lens.numel()), sigma, g, k
        a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().gakco_resident_create(ctx._h, _ptr(seqs), _ptr(lens), self.n_sv, sigma, g, k,
                                           a.ctypes.data_as(ctypes.c_void_p) if a is not None else None,
                                           float(bias), ctypes.byref(h)))
        self._h = h

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().gakco_resident_info(self._h, None, None, None, None, ctypes.byref(b)))
        return b.value

    def rows(self, q_seqs, q_lens, want_nm: bool = False, ctx: Context | None = None):
        """K-hat rows [n_q, n_sv] f64, decision values [n_q] f64, N_m rows if asked."""
        ctx = ctx or self.ctx
        q_seqs, q_lens = _dev_inputs(q_seqs, q_lens, ctx.device)
        n_q, M = int(q_lens.numel()), self.g - self.k
        K = torch.empty((n_q, self.n_sv), dtype=torch.float64, device=ctx.device)
        dec = torch.empty(n_q, dtype=torch.float64, device=ctx.device)
        Nm = torch.empty((M + 1, n_q, self.n_sv), dtype=torch.int64, device=ctx.device) if want_nm else None
        _check(lib().gakco_rows(ctx._h, self._h, _ptr(q_seqs), _ptr(q_lens), n_q, _ptr(K), _ptr(Nm), _ptr(dec),
                                _stream(ctx.device)))
        out = {"K": K, "decision": dec}
        if want_nm:
            out["Nm"] = Nm
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().gakco_resident_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IncrementalGram:
    """A normalised Gram matrix that grows by appended batches of sequences;
    `append` returns the new (N+n) x (N+n) matrix (device f64)."""

    def __init__(self, ctx: Context, sigma: int, g: int, k: int):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().gakco_incr_create(ctx._h, sigma, g, k, ctypes.byref(h)))
        self._h = h
        self.K = None

    @property
    def N(self) -> int:
        n = ctypes.c_int64()
        _check(lib().gakco_incr_info(self._h, ctypes.byref(n), None))
        return n.value

    def append(self, seqs, lens):
        seqs, lens = _dev_inputs(seqs, lens, self.ctx.device)
        n_new = int(lens.numel())
        Nt = self.N + n_new
        out = torch.empty((Nt, Nt), dtype=torch.float64, device=self.ctx.device)
        _check(lib().gakco_incr_append(self._h, _ptr(seqs), _ptr(lens), n_new, _ptr(self.K), _ptr(out),
                                       _stream(self.ctx.device)))
        self.K = out
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().gakco_incr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over a resident set (host queries)."""

    def __init__(self, resident: Resident, max_batch: int = 256, n_streams: int = 2, hbm_budget: int = 0, device: int = 0):
        self.res = resident
        h = ctypes.c_void_p()
        _check(lib().gakco_server_create(resident._h, device, max_batch, n_streams, hbm_budget, ctypes.byref(h)))
        self._h = h

    def set_param(self, name: str, value: int):
        """A tuning parameter on every worker (waits until no batch runs)."""
        _check(lib().gakco_server_set_param(self._h, name.encode(), int(value)))

    def submit(self, q, tag: int):
        import numpy as np
        q = np.ascontiguousarray(q, dtype=np.int8)
        _check(lib().gakco_server_submit(self._h, q.ctypes.data_as(ctypes.c_void_p) if q.size else None,
                                         int(q.size), int(tag)))

    def cancel(self, tag: int) -> bool:
        rc = lib().gakco_server_cancel(self._h, int(tag))
        if rc == EAGAIN:
            return False
        _check(rc)
        return True

    def poll(self, max_results: int = 64, wait_us: int = 1000, rows: bool = True):
        """Finished requests (dicts); with rows=False the K rows are not copied
        out (their "K_row" is None)."""
        import numpy as np
        arr = (Result * max_results)()
        n = ctypes.c_int32()
        rc = lib().gakco_server_poll(self._h, arr, max_results, ctypes.byref(n), wait_us)
        if rc not in (OK, EAGAIN):
            _check(rc)
        out = []
        for i in range(n.value):
            r = arr[i]
            row = None
            if r.K_row and rows:
                row = np.ctypeslib.as_array(ctypes.cast(r.K_row, ctypes.POINTER(ctypes.c_double)),
                                            shape=(self.res.n_sv,)).copy()
            out.append({"tag": r.tag, "status": r.status, "decision": r.decision, "K_row": row,
                        "t_submit": r.t_submit, "t_start": r.t_start, "t_done": r.t_done,
                        "batch_size": r.batch_size})
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().gakco_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 512 << 20


def gram_noalloc(seqs, lens, N: int, sigma: int, g: int, k: int, K=None, Nm=None, Cm=None, device: int = 0):
    """gakco_gram_noalloc on device tensors already in place: the library
    allocates no device memory (its scratch is a fixed device array)."""
    with torch.cuda.device(device):
        _check(lib().gakco_gram_noalloc(_ptr(seqs), _ptr(lens), int(N), int(sigma), int(g), int(k), _ptr(K), _ptr(Nm),
                                        _ptr(Cm), _stream(device)))


def version() -> str:
    return lib().gakco_version().decode()
