"""Python binding of the gfx950 C ABI (``include/lpcc.h``): argument marshalling only.

Every step of encoding, decoding and probability evaluation runs in the HIP
library ``liblpcc.so``; this module only passes pointers and sizes.  Inputs
may be numpy arrays (host memory) or torch tensors (host or device); device
tensors are passed by pointer, so the library reads them in place.  There is
no fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpcc.so")

OK, E_INVAL, E_CAPACITY, E_CORRUPT, E_MODEL, E_DEVICE, E_NOMEM = 0, -1, -2, -3, -4, -5, -6
_NAMES = {E_INVAL: "LPCC_E_INVAL", E_CAPACITY: "LPCC_E_CAPACITY", E_CORRUPT: "LPCC_E_CORRUPT",
          E_MODEL: "LPCC_E_MODEL", E_DEVICE: "LPCC_E_DEVICE", E_NOMEM: "LPCC_E_NOMEM"}



class Job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("model", ctypes.c_int), ("inp", ctypes.c_void_p),
                ("n_points", ctypes.c_int64), ("in_len", ctypes.c_size_t), ("out", ctypes.c_void_p),
                ("out_cap", ctypes.c_size_t), ("t_arrival_ns", ctypes.c_int64), ("chunk_log2", ctypes.c_int)]


class Done(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int), ("kind", ctypes.c_int),
                ("out_len", ctypes.c_size_t), ("n_points", ctypes.c_int64), ("t_arrival_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64), ("batch", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("mpts_per_s", ctypes.c_double), ("completed", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64), ("bytes_in_use", ctypes.c_size_t),
                ("bytes_budget", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t)]


class LpccError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{_NAMES.get(code, code)} {msg}".strip())
        self.code = code


_lib = None


def lib():
    """Load liblpcc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2603_25260_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int
        L.lpcc_model_load.argtypes = [vp, sz, i32, ctypes.POINTER(vp)]
        L.lpcc_model_free.argtypes = [vp]
        L.lpcc_model_free.restype = None
        L.lpcc_model_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_uint32)]
        L.lpcc_make_weights.argtypes = [ctypes.c_uint64, i32, i32, i32, i32, vp, sz, ctypes.POINTER(sz)]
        L.lpcc_ctx_create.argtypes = [i32, vp, sz, ctypes.POINTER(vp)]
        L.lpcc_ctx_workspace.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.lpcc_ctx_free.argtypes = [vp]
        L.lpcc_ctx_free.restype = None
        L.lpcc_last_error.argtypes = [vp]
        L.lpcc_last_error.restype = ctypes.c_char_p
        L.lpcc_encode_frame.argtypes = [vp, vp, vp, i64, i32, vp, sz, ctypes.POINTER(sz)]
        L.lpcc_encode_frame_noalloc.argtypes = [vp, vp, vp, i64, i32, vp, sz, ctypes.POINTER(sz)]
        L.lpcc_decode_frame.argtypes = [vp, vp, vp, sz, vp, i64, ctypes.POINTER(i64)]
        L.lpcc_level_probs.argtypes = [vp, vp, vp, i64, i32, vp, i64, ctypes.POINTER(i64)]
        L.lpcc_peek_header.argtypes = [vp, sz, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(sz)]
        L.lpcc_encode_batch.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp, vp, vp]
        L.lpcc_decode_batch.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp]
        L.lpcc_timing_enable.argtypes = [vp, ctypes.c_char_p]
        L.lpcc_timing_read.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(i64)]
        L.lpcc_softmax_table.argtypes = [vp]
        L.lpcc_requant_bounds.argtypes = [i32, i32, i32, i32, vp]
        L.lpcc_ctx_set_tiling.argtypes = [vp, i32]
        L.lpcc_ctx_set_base_depth.argtypes = [vp, i32]
        L.lpcc_ctx_set_kmap_mode.argtypes = [vp, i32]
        L.lpcc_ctx_set_graphs.argtypes = [vp, i32]
        L.lpcc_ctx_graph_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.lpcc_ctx_tuning.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.lpcc_ctx_set_tuning.argtypes = [vp, vp, i32]
        L.lpcc_server_create.argtypes = [i32, vp, i32, i32, i32, sz, ctypes.POINTER(vp)]
        L.lpcc_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
        L.lpcc_server_poll.argtypes = [vp, ctypes.POINTER(Done), i32, ctypes.POINTER(i32), i32]
        L.lpcc_server_drain.argtypes = [vp]
        L.lpcc_server_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.lpcc_server_free.argtypes = [vp]
        L.lpcc_server_free.restype = None
        _lib = L
    return _lib


def _ptr(a):
    """(pointer, keepalive) of a numpy array or torch tensor."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        a = np.ascontiguousarray(a)
        return a.ctypes.data, a
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            a = a.contiguous()
        return a.data_ptr(), a
    if isinstance(a, (bytes, bytearray)):
        b = np.frombuffer(a, np.uint8) if len(a) else np.zeros(1, np.uint8)
        return b.ctypes.data, b
    raise TypeError(type(a))


def _is_torch(a):
    return hasattr(a, "data_ptr") and hasattr(a, "device")


def softmax_table() -> np.ndarray:
    """The library's integer exponent table (host computation)."""
    out = np.zeros(256, np.int32)
    _check(lib().lpcc_softmax_table(out.ctypes.data))
    return out


def requant_bounds(m_pos: int, m_neg: int, r: int, z_out: int):
    """(m_pos, m_neg, a_lo, a_hi, rq24) of a requantisation as the kernels
    use it (host computation)."""
    out = np.zeros(5, np.int32)
    _check(lib().lpcc_requant_bounds(m_pos, m_neg, r, z_out, out.ctypes.data))
    return tuple(int(v) for v in out)


W_NO_XFP, W_ZERO_POINTS, W_SHARED = 1, 2, 4


def make_weights(seed: int, C: int, D: int, n_deep: int, *, xfp: bool = True, zero_points: bool = False,
                 shared: bool = False) -> bytes:
    """Seeded random-init weight blob, built by the library (host only)."""
    flags = (0 if xfp else W_NO_XFP) | (W_ZERO_POINTS if zero_points else 0) | (W_SHARED if shared else 0)
    n = ctypes.c_size_t()
    st = lib().lpcc_make_weights(seed, C, D, n_deep, flags, None, 0, ctypes.byref(n))
    if st not in (OK, E_CAPACITY):
        _check(st)
    buf = np.zeros(n.value, np.uint8)
    _check(lib().lpcc_make_weights(seed, C, D, n_deep, flags, buf.ctypes.data, n.value, ctypes.byref(n)))
    return buf.tobytes()


def peek_header(bs):
    """(D, points, max_workspace) of a host stream (max_workspace is 0 when
    the given bytes do not reach the depth counts)."""
    b = np.frombuffer(bytes(bs), np.uint8)
    D, npts, ws = ctypes.c_int(), ctypes.c_int64(), ctypes.c_size_t()
    _check(lib().lpcc_peek_header(b.ctypes.data, len(b), ctypes.byref(D), ctypes.byref(npts), ctypes.byref(ws)))
    return D.value, npts.value, ws.value


def _check(st, ctx=None):
    if st != OK:
        msg = ""
        if ctx is not None:
            m = lib().lpcc_last_error(ctx)
            msg = m.decode() if m else ""
        raise LpccError(st, msg)


class Model:
    def __init__(self, blob: bytes, device: int = 0):
        self._blob = np.frombuffer(blob, np.uint8).copy()
        h = ctypes.c_void_p()
        _check(lib().lpcc_model_load(self._blob.ctypes.data, len(blob), device, ctypes.byref(h)))
        self.handle = h
        C, D, nd, bid = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_uint32()
        _check(lib().lpcc_model_info(h, ctypes.byref(C), ctypes.byref(D), ctypes.byref(nd), ctypes.byref(bid)))
        self.C, self.D, self.n_deep, self.blob_id = C.value, D.value, nd.value, bid.value

    def close(self):
        if self.handle:
            lib().lpcc_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Device, stream and workspace.  ``stream`` is a hipStream_t handle (int)
    or None; with torch, pass ``torch.cuda.current_stream().cuda_stream``."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        _check(lib().lpcc_ctx_create(device, ctypes.c_void_p(stream) if stream else None, hbm_budget,
                                     ctypes.byref(h)))
        self.handle = h

    def workspace(self):
        """(bytes held now, most bytes held so far) of device workspace."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().lpcc_ctx_workspace(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        if self.handle:
            lib().lpcc_ctx_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tile shapes of the GEMM-type kernels: 0 autotunes, 1/2/4 fixes the
    # number of 16-row blocks per wave
    def set_tiling(self, rb: int):
        _check(lib().lpcc_ctx_set_tiling(self.handle, int(rb)), self.handle)

    # -- base geometry: depths below B coded from their own code counts
    def set_base_depth(self, base: int):
        _check(lib().lpcc_ctx_set_base_depth(self.handle, int(base)), self.handle)

    # -- neighbour tables: 0 derives each depth's from its parent depth's (a
    # hash at the first convolved depth only), 1 hashes every convolved depth
    def set_kmap_mode(self, mode: int):
        _check(lib().lpcc_ctx_set_kmap_mode(self.handle, int(mode)), self.handle)

    # -- graph mode: launch batches captured into HIP graphs and replayed
    def set_graphs(self, on: bool):
        _check(lib().lpcc_ctx_set_graphs(self.handle, 1 if on else 0), self.handle)

    def graph_stats(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lpcc_ctx_graph_stats(self.handle, ctypes.byref(a), ctypes.byref(b)), self.handle)
        return {"instantiated": a.value, "updated": b.value}

    def tuning(self):
        """Autotuner table: dicts with kind ('gemm'/'up'), mode, cin, cout,
        log2_rows and the chosen rb (0 while undecided)."""
        n = ctypes.c_int32()
        _check(lib().lpcc_ctx_tuning(self.handle, None, 0, ctypes.byref(n)), self.handle)
        buf = (ctypes.c_int32 * (6 * max(n.value, 1)))()
        _check(lib().lpcc_ctx_tuning(self.handle, buf, n.value, ctypes.byref(n)), self.handle)
        out = []
        for k in range(n.value):
            v = buf[6 * k:6 * k + 6]
            out.append({"kind": "up" if v[0] else "gemm", "mode": v[1], "cin": v[2], "cout": v[3],
                        "log2_rows": v[4], "rb": v[5]})
        return out

    def set_tuning(self, table):
        """Import an autotuner table in the format `tuning` returns: each
        class then uses its recorded variant without timing candidates."""
        rows = [[1 if t["kind"] == "up" else 0, t["mode"], t["cin"], t["cout"], t["log2_rows"], t["rb"]]
                for t in table]
        buf = (ctypes.c_int32 * (6 * max(len(rows), 1)))(*[int(x) for r in rows for x in r])
        _check(lib().lpcc_ctx_set_tuning(self.handle, buf, len(rows)), self.handle)

    # -- timing of one kernel family (HIP events on the context's stream)
    def timing_enable(self, family: str):
        _check(lib().lpcc_timing_enable(self.handle, family.encode()))

    def timing_read(self):
        n, ms, u = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().lpcc_timing_read(self.handle, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(u)), self.handle)
        return n.value, ms.value, u.value


def _n_points(xyz):
    return int(xyz.shape[0]) if xyz is not None else 0


def encode_frame(ctx: Context, model: Model, xyz, chunk_log2: int = 10, out=None):
    """Bitstream of one frame.  With ``out`` (a uint8 buffer, host or device)
    the stream is written there and its length returned; otherwise bytes."""
    p, keep = _ptr(xyz)
    n = _n_points(xyz)
    L = lib()
    if out is None:
        cap = 64 + 4 * model.D + 4 * max(n, 1) + 16 * model.D
        buf = np.zeros(cap, np.uint8)
        ln = ctypes.c_size_t()
        st = L.lpcc_encode_frame(ctx.handle, model.handle, p, n, chunk_log2, buf.ctypes.data, cap, ctypes.byref(ln))
        if st == E_CAPACITY:
            buf = np.zeros(ln.value, np.uint8)
            st = L.lpcc_encode_frame(ctx.handle, model.handle, p, n, chunk_log2, buf.ctypes.data, ln.value,
                                     ctypes.byref(ln))
        _check(st, ctx.handle)
        return buf[:ln.value].tobytes()
    op, okeep = _ptr(out)
    ln = ctypes.c_size_t()
    cap = out.numel() if _is_torch(out) else out.size
    _check(L.lpcc_encode_frame(ctx.handle, model.handle, p, n, chunk_log2, op, cap, ctypes.byref(ln)), ctx.handle)
    return ln.value


def encode_frame_noalloc(ctx: Context, model: Model, xyz, out, chunk_log2: int = 10) -> int:
    """Stream of one frame written into ``out`` (uint8, host or device) by the
    allocation-free entry point (static device workspace); returns its length."""
    p, keep = _ptr(xyz)
    op, okeep = _ptr(out)
    cap = out.numel() if _is_torch(out) else out.size
    ln = ctypes.c_size_t()
    _check(lib().lpcc_encode_frame_noalloc(ctx.handle, model.handle, p, _n_points(xyz), chunk_log2, op, cap,
                                           ctypes.byref(ln)), ctx.handle)
    return ln.value


def decode_frame(ctx: Context, model: Model, bs, length=None, out=None):
    """Voxel coordinates [N, 3] int32 in Morton order.  ``bs`` is bytes, a
    numpy uint8 array or a torch uint8 tensor (host or device)."""
    p, keep = _ptr(bs)
    ln = length if length is not None else (bs.numel() if _is_torch(bs) else len(bs))
    L = lib()
    nout = ctypes.c_int64()
    if out is None:
        D, npts = ctypes.c_int(), ctypes.c_int64()
        if _is_torch(bs) and bs.is_cuda:
            hdr = bs[:16].cpu().numpy()
            npts_v = int(hdr[12:16].view(np.uint32)[0])
        else:
            hb = np.frombuffer(bytes(bs[:16]) if not isinstance(bs, np.ndarray) else bs[:16].tobytes(), np.uint8)
            st = L.lpcc_peek_header(hb.ctypes.data, 16, ctypes.byref(D), ctypes.byref(npts), None)
            _check(st)
            npts_v = npts.value
        res = np.zeros((max(npts_v, 1), 3), np.int32)
        _check(L.lpcc_decode_frame(ctx.handle, model.handle, p, ln, res.ctypes.data, res.shape[0],
                                   ctypes.byref(nout)), ctx.handle)
        return res[:nout.value]
    op, okeep = _ptr(out)
    cap = out.shape[0]
    _check(L.lpcc_decode_frame(ctx.handle, model.handle, p, ln, op, cap, ctypes.byref(nout)), ctx.handle)
    return nout.value


def level_probs(ctx: Context, model: Model, xyz, level: int, out=None):
    """CDF rows int32 [N_level, 256] of one depth (the encoder's model output)."""
    p, keep = _ptr(xyz)
    n = _n_points(xyz)
    L = lib()
    nn = ctypes.c_int64()
    if out is None:
        st = L.lpcc_level_probs(ctx.handle, model.handle, p, n, level, None, 0, ctypes.byref(nn))
        if st not in (OK, E_CAPACITY):
            _check(st, ctx.handle)
        res = np.zeros((max(nn.value, 1), 256), np.int32)
        _check(L.lpcc_level_probs(ctx.handle, model.handle, p, n, level, res.ctypes.data, res.shape[0],
                                  ctypes.byref(nn)), ctx.handle)
        return res[:nn.value]
    op, okeep = _ptr(out)
    _check(L.lpcc_level_probs(ctx.handle, model.handle, p, n, level, op, out.shape[0], ctypes.byref(nn)), ctx.handle)
    return nn.value


def encode_batch(ctx: Context, model: Model, frames, chunk_log2: int = 10, outs=None):
    """Encode several frames in shared launches.  Returns a list of bytes
    (or of lengths when device ``outs`` are given) and the status list."""
    nf = len(frames)
    ptrs, keep = [], []
    for x in frames:
        p, k = _ptr(x)
        ptrs.append(p or 0)
        keep.append(k)
    n = np.array([_n_points(x) for x in frames], np.int64)
    xp = (ctypes.c_void_p * nf)(*ptrs)
    status = np.zeros(nf, np.int32)
    lens = np.zeros(nf, np.uint64)
    L = lib()
    if outs is None:
        caps = np.array([64 + 4 * model.D + 4 * max(int(v), 1) + 16 * model.D for v in n], np.uint64)
        bufs = [np.zeros(int(c_), np.uint8) for c_ in caps]
        op = (ctypes.c_void_p * nf)(*[b.ctypes.data for b in bufs])
        st = L.lpcc_encode_batch(ctx.handle, model.handle, nf, xp, n.ctypes.data, chunk_log2, op, caps.ctypes.data,
                                 lens.ctypes.data, status.ctypes.data)
        if st == E_CAPACITY and all(v in (OK, E_CAPACITY) for v in status):
            # the required sizes were written back: retry with exact buffers
            caps = lens.copy()
            bufs = [np.zeros(max(int(c_), 1), np.uint8) for c_ in caps]
            op = (ctypes.c_void_p * nf)(*[b.ctypes.data for b in bufs])
            st = L.lpcc_encode_batch(ctx.handle, model.handle, nf, xp, n.ctypes.data, chunk_log2, op,
                                     caps.ctypes.data, lens.ctypes.data, status.ctypes.data)
        if st not in (OK, E_CAPACITY):
            _check(st, ctx.handle)
        return [bufs[i][:int(lens[i])].tobytes() if status[i] == OK else None for i in range(nf)], status.tolist()
    okeep = [_ptr(o) for o in outs]
    op = (ctypes.c_void_p * nf)(*[k[0] for k in okeep])
    caps = np.array([o.numel() if _is_torch(o) else o.size for o in outs], np.uint64)
    st = L.lpcc_encode_batch(ctx.handle, model.handle, nf, xp, n.ctypes.data, chunk_log2, op, caps.ctypes.data,
                             lens.ctypes.data, status.ctypes.data)
    if st not in (OK, E_CAPACITY):
        _check(st, ctx.handle)
    return [int(v) for v in lens], status.tolist()


def decode_batch(ctx: Context, model: Model, streams, lengths=None, outs=None):
    nf = len(streams)
    ptrs, keep = [], []
    for x in streams:
        p, k = _ptr(x)
        ptrs.append(p)
        keep.append(k)
    if lengths is None:
        lengths = [(s.numel() if _is_torch(s) else len(s)) for s in streams]
    ln = np.array(lengths, np.uint64)
    bp = (ctypes.c_void_p * nf)(*ptrs)
    status = np.zeros(nf, np.int32)
    nout = np.zeros(nf, np.int64)
    L = lib()
    if outs is None:
        caps = []
        for s_ in streams:
            hb = (s_[:16].cpu().numpy() if _is_torch(s_) else np.frombuffer(bytes(s_[:16]), np.uint8))
            caps.append(max(1, int(np.asarray(hb[12:16], np.uint8).view(np.uint32)[0])) if len(hb) >= 16 else 1)
        res = [np.zeros((c_, 3), np.int32) for c_ in caps]
        op = (ctypes.c_void_p * nf)(*[r.ctypes.data for r in res])
        cp = np.array(caps, np.int64)
        st = L.lpcc_decode_batch(ctx.handle, model.handle, nf, bp, ln.ctypes.data, op, cp.ctypes.data,
                                 nout.ctypes.data, status.ctypes.data)
        if st not in (OK, E_CAPACITY, E_CORRUPT, E_MODEL):
            _check(st, ctx.handle)
        return [res[i][:nout[i]] if status[i] == OK else None for i in range(nf)], status.tolist()
    okeep = [_ptr(o) for o in outs]
    op = (ctypes.c_void_p * nf)(*[k[0] for k in okeep])
    cp = np.array([o.shape[0] for o in outs], np.int64)
    st = L.lpcc_decode_batch(ctx.handle, model.handle, nf, bp, ln.ctypes.data, op, cp.ctypes.data, nout.ctypes.data,
                             status.ctypes.data)
    if st not in (OK, E_CAPACITY, E_CORRUPT, E_MODEL):
        _check(st, ctx.handle)
    return nout.tolist(), status.tolist()


class Server:
    """Continuous-batching server (see lpcc_server_* in include/lpcc.h).
    Buffers handed to ``submit`` must stay alive until the job is polled."""

    def __init__(self, models, device: int = 0, slots: int = 4, max_batch: int = 4, hbm_budget: int = 0):
        self.models = list(models)
        arr = (ctypes.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        h = ctypes.c_void_p()
        _check(lib().lpcc_server_create(device, arr, len(self.models), slots, max_batch, hbm_budget,
                                        ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, kind: int, model: int, inp, out, *, n_points=0, in_len=0, chunk_log2=8, t_arrival_ns=0):
        ip, ik = _ptr(inp)
        op, ok = _ptr(out)
        if kind == 0:
            n_points = n_points or _n_points(inp)
            cap = out.numel() if _is_torch(out) else out.size
        else:
            in_len = in_len or (inp.numel() if _is_torch(inp) else len(inp))
            cap = out.shape[0]
        j = Job(kind, model, ip, n_points, in_len, op, cap, t_arrival_ns, chunk_log2)
        t = ctypes.c_uint64()
        _check(lib().lpcc_server_submit(self.handle, ctypes.byref(j), ctypes.byref(t)))
        self._keep[t.value] = (ik, ok)
        return t.value

    def poll(self, max_n: int = 256, wait_ms: int = 0):
        buf = (Done * max_n)()
        n = ctypes.c_int()
        _check(lib().lpcc_server_poll(self.handle, buf, max_n, ctypes.byref(n), wait_ms))
        out = []
        for i in range(n.value):
            d = buf[i]
            self._keep.pop(d.ticket, None)
            out.append({"ticket": d.ticket, "status": d.status, "kind": d.kind, "out_len": d.out_len,
                        "n_points": d.n_points, "t_arrival_ns": d.t_arrival_ns, "t_start_ns": d.t_start_ns,
                        "t_done_ns": d.t_done_ns, "batch": d.batch})
        return out

    def drain(self):
        _check(lib().lpcc_server_drain(self.handle))

    def stats(self):
        st = Stats()
        _check(lib().lpcc_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in Stats._fields_}

    def close(self):
        if self.handle:
            lib().lpcc_server_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
