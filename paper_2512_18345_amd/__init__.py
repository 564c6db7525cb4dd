"""Python binding of libckks.so, the gfx950 RNS-CKKS key-switching library.

Argument marshalling only: every function below forwards to the C entry
point of the same name (declared in include/ckks.h); all arithmetic runs in
the library's HIP kernels.  Tensors are device tensors (torch, any 32-bit
integer dtype, contiguous); PyTorch supplies device memory and streams.
There is no fallback: if the library is not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

__all__ = [
    "CkksError", "lib", "Context", "OP",
    "ckks_ctx_create", "ckks_ctx_destroy", "ckks_workspace_bytes",
    "ckks_ntt", "ckks_intt", "ckks_automorph", "ckks_tensor", "ckks_modup",
    "ckks_inner_product", "ckks_moddown", "ckks_keyswitch", "ckks_hmult", "ckks_hmult_noalloc",
    "ckks_hrot", "ckks_hrot_hoisted", "ckks_rescale", "ckks_trace_begin", "ckks_trace_end", "STAGE",
    "JOB", "ckks_job", "ckks_batch_create", "ckks_batch_launch", "ckks_batch_device_bytes",
    "ckks_batch_destroy", "ckks_batch_plan", "ckks_batch_get_plan", "ckks_batch_set_plan",
    "ckks_batch_tune", "ckks_batch_tune_log", "ckks_stats", "ckks_server_create", "ckks_server_submit",
    "ckks_server_poll", "ckks_server_drain", "ckks_server_set_accounting", "ckks_server_stats", "ckks_server_times",
    "ckks_server_destroy", "ckks_pmult_sum", "ckks_pmult_sums", "ckks_hrot_many", "ckks_add", "ckks_schedule", "ckks_ctx_get_schedule",
    "ckks_ctx_set_schedule", "ckks_ctx_tune", "ckks_batch_get_schedule", "ckks_batch_set_schedule",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libckks.so")

OP = dict(NTT=0, MODUP=1, MODDOWN=2, KEYSWITCH=3, HMULT=4, HROT=5, RESCALE=6, HROT_HOISTED=7)
STAGE = dict(INTT_BLOCKS=1, INTT_COLS=2, BCONV_UP=3, NTT_COLS_UP=4, NTT_IP=5, INTT_COLS_P=6,
             BCONV_DOWN=7, NTT_COLS_DOWN=8, NTT_COMBINE=9, RESCALE_NTT=10, NTT_IP_P=11)


class CkksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ckks error {code}: {msg}")
        self.code = code


JOB = dict(KEYSWITCH=0, HMULT=1, HROT=2, RESCALE=3)


class ckks_job(ctypes.Structure):
    """Mirror of struct ckks_job (include/ckks.h)."""
    _fields_ = [("op", ctypes.c_int), ("L", ctypes.c_int), ("rot", ctypes.c_int),
                ("reserved", ctypes.c_int), ("in0", ctypes.c_void_p), ("in1", ctypes.c_void_p),
                ("key", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class ckks_schedule(ctypes.Structure):
    """Mirror of struct ckks_schedule (include/ckks.h)."""
    _fields_ = [("bconv_up_rows", ctypes.c_int), ("bconv_down_rows", ctypes.c_int),
                ("small_grid", ctypes.c_int), ("ntt_shape", ctypes.c_int)]

    def as_dict(self):
        return dict(bconv_up_rows=self.bconv_up_rows, bconv_down_rows=self.bconv_down_rows,
                    small_grid=self.small_grid, ntt_shape=self.ntt_shape)


class ckks_batch_plan(ctypes.Structure):
    """Mirror of struct ckks_batch_plan (include/ckks.h)."""
    _fields_ = [("jobs_per_launch", ctypes.c_int), ("streams", ctypes.c_int),
                ("split", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self):
        return dict(jobs_per_launch=self.jobs_per_launch, streams=self.streams, split=self.split)


class ckks_stats(ctypes.Structure):
    """Mirror of struct ckks_stats (include/ckks.h)."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("in_flight", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("ks_per_s", ctypes.c_double), ("budget_bytes", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_sz = ctypes.c_size_t

_SIGS = {
    "ckks_ctx_create": [ctypes.POINTER(_vp), _i, _vp, _i, _vp, _i, _i, _i],
    "ckks_ctx_destroy": [_vp],
    "ckks_ntt": [_vp, _vp, _i, _i, _vp],
    "ckks_intt": [_vp, _vp, _i, _i, _vp],
    "ckks_automorph": [_vp, _vp, _vp, _i, _i, _vp],
    "ckks_tensor": [_vp, _vp, _vp, _i, _vp, _vp],
    "ckks_modup": [_vp, _vp, _i, _vp, _vp, _sz, _vp],
    "ckks_inner_product": [_vp, _vp, _i, _vp, _vp, _vp],
    "ckks_moddown": [_vp, _vp, _i, _vp, _vp, _sz, _vp],
    "ckks_keyswitch": [_vp, _vp, _i, _vp, _vp, _vp, _sz, _vp],
    "ckks_hmult": [_vp, _vp, _vp, _i, _vp, _vp, _vp, _sz, _vp],
    "ckks_hmult_noalloc": [_vp, _vp, _vp, _i, _vp, _vp, _vp],
    "ckks_hrot": [_vp, _vp, _i, _i, _vp, _vp, _vp, _sz, _vp],
    "ckks_hrot_hoisted": [_vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _sz, _vp],
    "ckks_rescale": [_vp, _vp, _i, _vp, _vp, _sz, _vp],
    "ckks_trace_begin": [_vp, _i, _i],
    "ckks_batch_create": [_vp, _vp, _i, _i, ctypes.POINTER(_vp)],
    "ckks_batch_launch": [_vp, _vp],
    "ckks_batch_destroy": [_vp],
    "ckks_batch_get_plan": [_vp, _vp],
    "ckks_ctx_get_schedule": [_vp, _vp],
    "ckks_ctx_set_schedule": [_vp, _vp],
    "ckks_ctx_tune": [_vp, _i, _i, _vp, _vp, _vp],
    "ckks_batch_set_plan": [_vp, _vp],
    "ckks_batch_get_schedule": [_vp, _vp],
    "ckks_batch_set_schedule": [_vp, _vp],
    "ckks_batch_tune": [_vp, _i, _vp, _vp, _vp],
    "ckks_batch_tune_log": [_vp, _vp, _vp, _i, ctypes.POINTER(_i)],
    "ckks_pmult_sum": [_vp, _vp, _vp, _i, _i, _vp, _vp],
    "ckks_pmult_sums": [_vp, _vp, _i, _vp, _i, _i, _vp, _vp],
    "ckks_hrot_many": [_vp, _vp, _i, _vp, _vp, _vp, _i, _vp, _sz, _vp],
    "ckks_add": [_vp, _vp, _vp, _i, _vp, _vp],
    "ckks_server_create": [_vp, _i, _sz, _i, ctypes.POINTER(_vp)],
    "ckks_server_submit": [_vp, _i, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)],
    "ckks_server_poll": [_vp, ctypes.c_uint64, ctypes.POINTER(_i)],
    "ckks_server_drain": [_vp],
    "ckks_server_set_accounting": [_vp, _i],
    "ckks_server_stats": [_vp, _vp],
    "ckks_server_times": [_vp, ctypes.c_uint64, _i, _vp, _vp],
    "ckks_server_destroy": [_vp],
    "ckks_trace_end": [_vp, _vp, ctypes.POINTER(_i)],
}


def lib() -> ctypes.CDLL:
    """Load libckks.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2512_18345_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _i
        L.ckks_last_error.restype = ctypes.c_char_p
        L.ckks_last_error.argtypes = []
        L.ckks_workspace_bytes.restype = _sz
        L.ckks_workspace_bytes.argtypes = [_vp, _i, _i]
        L.ckks_batch_device_bytes.restype = _sz
        L.ckks_batch_device_bytes.argtypes = [_vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise CkksError(rc, lib().ckks_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device address of a tensor (or an int address / None)."""
    if t is None or isinstance(t, int):
        return t
    if t.dtype.itemsize != 4 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous 32-bit integer device tensor")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ws(ws):
    if ws is None:
        return None, 0
    return _ptr(ws), ws.numel() * ws.element_size()


def _u32_array(vals: Sequence[int]):
    arr = (ctypes.c_uint32 * len(vals))(*[int(v) for v in vals])
    return arr


# ----- one wrapper per C entry point -----------------------------------------

def ckks_ctx_create(logN: int, q: Sequence[int], p: Sequence[int], dnum: int, device: int = 0) -> int:
    h = _vp()
    qa, pa = _u32_array(q), _u32_array(p)
    _check(lib().ckks_ctx_create(ctypes.byref(h), logN, ctypes.cast(qa, _vp), len(q),
                                 ctypes.cast(pa, _vp), len(p), dnum, device))
    return h.value


def ckks_ctx_destroy(ctx: int) -> None:
    _check(lib().ckks_ctx_destroy(ctx))


def ckks_workspace_bytes(ctx: int, op: int, L: int) -> int:
    return int(lib().ckks_workspace_bytes(ctx, op, L))


def ckks_ntt(ctx, a, L, with_P=False, stream=None):
    _check(lib().ckks_ntt(ctx, _ptr(a), L, int(bool(with_P)), _stream(stream)))


def ckks_intt(ctx, a, L, with_P=False, stream=None):
    _check(lib().ckks_intt(ctx, _ptr(a), L, int(bool(with_P)), _stream(stream)))


def ckks_automorph(ctx, inp, out, rows, rot, stream=None):
    _check(lib().ckks_automorph(ctx, _ptr(inp), _ptr(out), rows, rot, _stream(stream)))


def ckks_tensor(ctx, ct1, ct2, L, out, stream=None):
    _check(lib().ckks_tensor(ctx, _ptr(ct1), _ptr(ct2), L, _ptr(out), _stream(stream)))


def ckks_modup(ctx, d, L, out, ws=None, stream=None):
    w, nb = _ws(ws)
    _check(lib().ckks_modup(ctx, _ptr(d), L, _ptr(out), w, nb, _stream(stream)))


def ckks_inner_product(ctx, M, L, evk, acc, stream=None):
    _check(lib().ckks_inner_product(ctx, _ptr(M), L, _ptr(evk), _ptr(acc), _stream(stream)))


def ckks_moddown(ctx, inp, L, out, ws=None, stream=None):
    w, nb = _ws(ws)
    _check(lib().ckks_moddown(ctx, _ptr(inp), L, _ptr(out), w, nb, _stream(stream)))


def ckks_keyswitch(ctx, d, L, evk, out, ws=None, stream=None):
    w, nb = _ws(ws)
    _check(lib().ckks_keyswitch(ctx, _ptr(d), L, _ptr(evk), _ptr(out), w, nb, _stream(stream)))


def ckks_hmult(ctx, ct1, ct2, L, rlk, out, ws=None, stream=None):
    w, nb = _ws(ws)
    _check(lib().ckks_hmult(ctx, _ptr(ct1), _ptr(ct2), L, _ptr(rlk), _ptr(out), w, nb, _stream(stream)))


def ckks_hmult_noalloc(ctx, ct1, ct2, L, rlk, out, stream=None):
    _check(lib().ckks_hmult_noalloc(ctx, _ptr(ct1), _ptr(ct2), L, _ptr(rlk), _ptr(out), _stream(stream)))


def ckks_hrot(ctx, ct, L, rot, rotk, out, ws=None, stream=None):
    w, nb = _ws(ws)
    _check(lib().ckks_hrot(ctx, _ptr(ct), L, rot, _ptr(rotk), _ptr(out), w, nb, _stream(stream)))


def ckks_hrot_hoisted(ctx, ct, L, rots, rotks, outs, ws=None, stream=None):
    n = len(rots)
    assert len(rotks) == n and len(outs) == n
    r = (ctypes.c_int * n)(*[int(v) for v in rots])
    k = (_vp * n)(*[_ptr(t) for t in rotks])
    o = (_vp * n)(*[_ptr(t) for t in outs])
    w, nb = _ws(ws)
    _check(lib().ckks_hrot_hoisted(ctx, _ptr(ct), L, ctypes.cast(r, _vp), n, ctypes.cast(k, _vp),
                                   ctypes.cast(o, _vp), w, nb, _stream(stream)))


def ckks_rescale(ctx, ct, L, out, ws=None, stream=None):
    w, nb = _ws(ws)
    _check(lib().ckks_rescale(ctx, _ptr(ct), L, _ptr(out), w, nb, _stream(stream)))


def ckks_batch_create(ctx, jobs, use_graph=True) -> int:
    """jobs: sequence of dicts or ckks_job; tensors are taken by device address."""
    arr = (ckks_job * len(jobs))()
    for i, j in enumerate(jobs):
        if isinstance(j, ckks_job):
            arr[i] = j
        else:
            arr[i] = ckks_job(int(j["op"]), int(j["L"]), int(j.get("rot", 0)), 0,
                              _ptr(j["in0"]), _ptr(j.get("in1")), _ptr(j.get("key")), _ptr(j["out"]))
    h = _vp()
    _check(lib().ckks_batch_create(ctx, ctypes.cast(arr, _vp), len(jobs), int(bool(use_graph)),
                                   ctypes.byref(h)))
    return h.value


def ckks_batch_launch(batch, stream=None):
    _check(lib().ckks_batch_launch(batch, _stream(stream)))


def ckks_batch_device_bytes(batch) -> int:
    return int(lib().ckks_batch_device_bytes(batch))


def ckks_batch_destroy(batch):
    _check(lib().ckks_batch_destroy(batch))


def ckks_batch_get_plan(batch) -> dict:
    p = ckks_batch_plan()
    _check(lib().ckks_batch_get_plan(batch, ctypes.cast(ctypes.byref(p), _vp)))
    return p.as_dict()


def ckks_batch_set_plan(batch, jobs_per_launch=0, streams=1, split=1):
    p = ckks_batch_plan(int(jobs_per_launch), int(streams), int(split), 0)
    _check(lib().ckks_batch_set_plan(batch, ctypes.cast(ctypes.byref(p), _vp)))


def ckks_ctx_get_schedule(ctx) -> dict:
    s = ckks_schedule()
    _check(lib().ckks_ctx_get_schedule(ctx, ctypes.cast(ctypes.byref(s), _vp)))
    return s.as_dict()


def ckks_ctx_set_schedule(ctx, bconv_up_rows=12, bconv_down_rows=6, small_grid=128, ntt_shape=0):
    s = ckks_schedule(int(bconv_up_rows), int(bconv_down_rows), int(small_grid), int(ntt_shape))
    _check(lib().ckks_ctx_set_schedule(ctx, ctypes.cast(ctypes.byref(s), _vp)))


def ckks_ctx_tune(ctx, L, reps=3, stream=None):
    """Autotune the context's kernel schedule at level L; returns (schedule dict, us per HMult)."""
    s = ckks_schedule()
    us = ctypes.c_float()
    _check(lib().ckks_ctx_tune(ctx, int(L), int(reps), _stream(stream),
                               ctypes.cast(ctypes.byref(s), _vp), ctypes.cast(ctypes.byref(us), _vp)))
    return s.as_dict(), float(us.value)


def ckks_batch_get_schedule(batch) -> dict:
    s = ckks_schedule()
    _check(lib().ckks_batch_get_schedule(batch, ctypes.cast(ctypes.byref(s), _vp)))
    return s.as_dict()


def ckks_batch_set_schedule(batch, bconv_up_rows=12, bconv_down_rows=6, small_grid=128, ntt_shape=0):
    s = ckks_schedule(int(bconv_up_rows), int(bconv_down_rows), int(small_grid), int(ntt_shape))
    _check(lib().ckks_batch_set_schedule(batch, ctypes.cast(ctypes.byref(s), _vp)))


def ckks_batch_tune_log(batch) -> list:
    """[(plan dict, microseconds per launch)] of the last ckks_batch_tune."""
    n = _i()
    _check(lib().ckks_batch_tune_log(batch, None, None, 0, ctypes.byref(n)))
    plans = (ckks_batch_plan * max(n.value, 1))()
    us = (ctypes.c_float * max(n.value, 1))()
    _check(lib().ckks_batch_tune_log(batch, ctypes.cast(plans, _vp), ctypes.cast(us, _vp), n.value,
                                     ctypes.byref(n)))
    return [(plans[i].as_dict(), float(us[i])) for i in range(n.value)]


def ckks_batch_tune(batch, reps=3, stream=None):
    """Autotune the batch's plan; returns (plan dict, microseconds per launch)."""
    p = ckks_batch_plan()
    us = ctypes.c_float()
    _check(lib().ckks_batch_tune(batch, int(reps), _stream(stream),
                                 ctypes.cast(ctypes.byref(p), _vp), ctypes.cast(ctypes.byref(us), _vp)))
    return p.as_dict(), float(us.value)


def ckks_pmult_sum(ctx, cts, pts, L, out, stream=None):
    n = len(cts)
    a = (_vp * n)(*[_ptr(t) for t in cts])
    b = (_vp * n)(*[_ptr(t) for t in pts])
    _check(lib().ckks_pmult_sum(ctx, ctypes.cast(a, _vp), ctypes.cast(b, _vp), n, L, _ptr(out),
                                _stream(stream)))


def ckks_hrot_many(ctx, cts, L, rots, rotks, outs, ws, stream=None):
    """outs[i] = HRot(cts[i], rots[i]) under rotks[i], one launch sequence; ws holds
    len(cts) times the HRot workspace."""
    n = len(cts)
    if len(rots) != n or len(rotks) != n or len(outs) != n:
        raise CkksError(-1, "hrot_many: one rotation, key and output per ciphertext")
    a = (_vp * n)(*[_ptr(t) for t in cts])
    r = (_i * n)(*[int(x) for x in rots])
    k = (_vp * n)(*[_ptr(t) for t in rotks])
    o = (_vp * n)(*[_ptr(t) for t in outs])
    w, nb = _ws(ws)
    _check(lib().ckks_hrot_many(ctx, ctypes.cast(a, _vp), L, ctypes.cast(r, _vp), ctypes.cast(k, _vp),
                                ctypes.cast(o, _vp), n, w, nb, _stream(stream)))


def ckks_pmult_sums(ctx, cts, pt_groups, L, outs, stream=None):
    """outs[g] = sum_b cts[b] * pt_groups[g][b]; every group has len(cts) plaintexts."""
    nb, ng = len(cts), len(pt_groups)
    if any(len(grp) != nb for grp in pt_groups) or len(outs) != ng:
        raise CkksError(-1, "pmult_sums: one plaintext per ciphertext in every group, one output per group")
    a = (_vp * nb)(*[_ptr(t) for t in cts])
    b = (_vp * (ng * nb))(*[_ptr(t) for grp in pt_groups for t in grp])
    o = (_vp * ng)(*[_ptr(t) for t in outs])
    _check(lib().ckks_pmult_sums(ctx, ctypes.cast(a, _vp), nb, ctypes.cast(b, _vp), ng, L, ctypes.cast(o, _vp),
                                 _stream(stream)))


def ckks_add(ctx, a, b, L, out, stream=None):
    _check(lib().ckks_add(ctx, _ptr(a), _ptr(b), L, _ptr(out), _stream(stream)))


def _job(j):
    if isinstance(j, ckks_job):
        return j
    return ckks_job(int(j["op"]), int(j["L"]), int(j.get("rot", 0)), 0, _ptr(j["in0"]),
                    _ptr(j.get("in1")), _ptr(j.get("key")), _ptr(j["out"]))


def ckks_server_create(ctxs, hbm_budget, max_slots) -> int:
    arr = (_vp * len(ctxs))(*ctxs)
    h = _vp()
    _check(lib().ckks_server_create(ctypes.cast(arr, _vp), len(ctxs), int(hbm_budget), int(max_slots),
                                    ctypes.byref(h)))
    return h.value


def ckks_server_submit(server, ctx_index, job, stream=None) -> int:
    """stream: where the job's inputs were produced (default: torch's current stream)."""
    j = _job(job)
    t = ctypes.c_uint64(0)
    _check(lib().ckks_server_submit(server, int(ctx_index), ctypes.cast(ctypes.byref(j), _vp),
                                    _stream(stream), ctypes.byref(t)))
    return t.value


def ckks_server_poll(server, ticket) -> bool:
    d = _i(0)
    _check(lib().ckks_server_poll(server, int(ticket), ctypes.byref(d)))
    return bool(d.value)


def ckks_server_drain(server):
    _check(lib().ckks_server_drain(server))


def ckks_server_set_accounting(server, whole_footprint):
    _check(lib().ckks_server_set_accounting(server, int(whole_footprint)))


def ckks_server_stats(server) -> dict:
    st = ckks_stats()
    _check(lib().ckks_server_stats(server, ctypes.cast(ctypes.byref(st), _vp)))
    return st.as_dict()


def ckks_server_times(server, first, n):
    a = (ctypes.c_double * max(n, 1))()
    b = (ctypes.c_double * max(n, 1))()
    _check(lib().ckks_server_times(server, int(first), int(n), ctypes.cast(a, _vp), ctypes.cast(b, _vp)))
    return [a[i] for i in range(n)], [b[i] for i in range(n)]


def ckks_server_destroy(server):
    _check(lib().ckks_server_destroy(server))


def ckks_trace_begin(ctx, stage, capacity):
    _check(lib().ckks_trace_begin(ctx, int(stage), int(capacity)))


def ckks_trace_end(ctx, capacity):
    """Returns the per-launch durations (ms) recorded since ckks_trace_begin."""
    buf = (ctypes.c_float * max(int(capacity), 1))()
    n = _i(0)
    _check(lib().ckks_trace_end(ctx, ctypes.cast(buf, _vp), ctypes.byref(n)))
    return [float(buf[i]) for i in range(n.value)]


class Context:
    """Owns a ckks_ctx for one ring degree; allocates workspaces with torch."""

    def __init__(self, logN: int, q: Sequence[int], p: Sequence[int], dnum: int, device: int = 0):
        self.logN, self.N = logN, 1 << logN
        self.q, self.p, self.dnum, self.device = list(q), list(p), dnum, device
        self.L_max, self.k = len(q), len(p)
        self.alpha = -(-self.L_max // dnum)
        self.handle = ckks_ctx_create(logN, q, p, dnum, device)

    @classmethod
    def from_spec(cls, spec, device: int = 0) -> "Context":
        return cls(spec.logN, spec.q, spec.p, spec.dnum, device)

    def beta(self, L: int) -> int:
        return -(-L // self.alpha)

    def workspace(self, op: str, L: int, count: int = 1):
        """Device workspace for `count` jobs of `op` at level L (count > 1: ckks_hrot_many)."""
        import torch
        nb = ckks_workspace_bytes(self.handle, OP[op], L) * count
        return torch.empty(max(nb // 4, 1), dtype=torch.int32, device=f"cuda:{self.device}")

    def close(self):
        if self.handle:
            ckks_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
