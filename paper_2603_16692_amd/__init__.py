"""MI355X (gfx950) CKKS hybrid KeySwitch: Python binding of libks.so.

The binding only marshals arguments: every step of the path runs in the HIP
kernels of ``libks.so`` (see ``include/ks.h`` for the contract of each
call). Tensors are torch device tensors of dtype int64 holding the uint64
residues (every residue is below 2^60, so the bit patterns agree); torch
supplies device memory and the HIP stream. There is no CPU fallback: if the
library is missing, importing this package raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libks.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)

KS_OK, KS_EINVAL, KS_ENULL, KS_EALIGN, KS_ENOMEM, KS_EUNSUP, KS_EHIP, KS_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_SCRATCH_BYTES = 128 << 20  # KS_NOALLOC_SCRATCH_BYTES: the static workspace of keyswitch_noalloc
KS_MAX_LIMBS = 128
KS_SET_P = -1
DSOB, DPOB, DSOC, DPOC, STAGED = 0, 1, 2, 3, 4
DATAFLOW_NAMES = {DSOB: "DSOB", DPOB: "DPOB", DSOC: "DSOC", DPOC: "DPOC", STAGED: "STAGED"}
PLAN_MFMA_BCONV = 1  # ks_plan.flags: BConv as an exact int8 product on the matrix cores
PLAN_SPLIT_STREAMS = 2  # ks_plan.flags: the two halves of a batch on two streams
PLAN_HOIST_FWD = 4  # ks_plan.flags (DPOB): the raised digits' forward block pass as a launch of its own


class Plan(ctypes.Structure):
    _fields_ = [("dataflow", ctypes.c_int), ("chunks", ctypes.c_int), ("log_r", ctypes.c_int),
                ("flags", ctypes.c_int), ("batch_tile", ctypes.c_int)]

    def __repr__(self):
        mx = ", mfma" if self.flags & PLAN_MFMA_BCONV else ""
        sp = ", split" if self.flags & PLAN_SPLIT_STREAMS else ""
        sp += ", hoist" if self.flags & PLAN_HOIST_FWD else ""
        tl = f", tile={self.batch_tile}" if self.batch_tile else ""
        return (f"Plan({DATAFLOW_NAMES.get(self.dataflow, self.dataflow)}, chunks={self.chunks}, "
                f"log_r={self.log_r}{mx}{sp}{tl})")

    def key(self):
        return (self.dataflow, self.chunks, self.log_r, self.flags, self.batch_tile)


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("log_n", ctypes.c_int), ("ell", ctypes.c_int), ("k", ctypes.c_int),
                ("alpha", ctypes.c_int), ("dnum", ctypes.c_int), ("ndig", ctypes.c_int), ("key_ell", ctypes.c_int),
                ("moduli", ctypes.c_uint64 * KS_MAX_LIMBS), ("psi", ctypes.c_uint64 * KS_MAX_LIMBS)]


_vp, _i, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
_lib.ks_params_create.argtypes = [_i, _i, _i, ctypes.POINTER(_vp)]
_lib.ks_params_at_level.argtypes = [_vp, _i, ctypes.POINTER(_vp)]
_lib.ks_params_destroy.argtypes = [_vp]
_lib.ks_params_destroy.restype = None
_lib.ks_params_info.argtypes = [_vp, ctypes.POINTER(Info)]
_lib.ks_workspace_bytes.argtypes = [_vp, _i, ctypes.POINTER(Plan), ctypes.POINTER(_sz)]
_lib.ks_default_plan.argtypes = [_vp, _i, ctypes.POINTER(Plan)]
_lib.ks_ntt.argtypes = [_vp, _vp, _i, _i, _i, _vp]
_lib.ks_intt.argtypes = [_vp, _vp, _i, _i, _i, _vp]
_lib.ks_bconv.argtypes = [_vp, _vp, _i, _vp, _i, _vp]
_lib.ks_modup.argtypes = [_vp, _vp, _vp, _i, _vp, _vp]
_lib.ks_keymult.argtypes = [_vp, _vp, _vp, _vp, _i, _vp]
_lib.ks_moddown.argtypes = [_vp, _vp, _vp, _i, _vp, _vp]
_lib.ks_keyswitch.argtypes = [_vp, _vp, _vp, _vp, _i, ctypes.POINTER(Plan), _vp, _vp]
_lib.ks_keyswitch_noalloc.argtypes = [_vp, _vp, _vp, _vp, _i, ctypes.POINTER(Plan), _vp]
_lib.ks_hmul.argtypes = [_vp, _vp, _vp, _vp, _vp, _i, ctypes.POINTER(Plan), _vp, _vp]
_lib.ks_hrot.argtypes = [_vp, _vp, _i, _vp, _vp, _i, ctypes.POINTER(Plan), _vp, _vp]
_lib.ks_eval_workspace_bytes.argtypes = [_vp, _i, ctypes.POINTER(Plan), ctypes.POINTER(_sz)]
_lib.ks_launch_count.argtypes = [_vp, _i, ctypes.POINTER(Plan)]
_lib.ks_modmul_rate.argtypes = [_vp, _i, _i, _i, _vp, _vp]
_lib.ks_modmul_chains.restype = _i
_lib.ks_copy_rate.argtypes = [_i, _i, _i, _vp, _vp, _sz, _vp]
_lib.ks_strerror.argtypes = [_i]
_lib.ks_strerror.restype = ctypes.c_char_p
_lib.ks_last_hip_error.restype = ctypes.c_char_p

_lib.ks_trace_begin.argtypes = [ctypes.POINTER(_vp), _i, ctypes.c_uint]
_lib.ks_trace_end.argtypes = [ctypes.POINTER(_i), _i]

_lib.ks_graph_create.argtypes = [_vp, _vp, _vp, _vp, _i, ctypes.POINTER(Plan), _vp, _vp, ctypes.POINTER(_vp)]
_lib.ks_graph_launch.argtypes = [_vp, _vp]
_lib.ks_graph_destroy.argtypes = [_vp]
_lib.ks_graph_destroy.restype = None

KIND_NAMES = ["intt_d_blocks", "modup_cols", "keymult_blocks", "moddown_cols", "moddown_blocks", "ext_blocks",
              "pblocks_inv", "copy_digits", "keymult", "bconv", "ntt", "eval"]

EXPORTED = ["ks_params_create", "ks_params_destroy", "ks_params_at_level", "ks_params_info", "ks_workspace_bytes",
            "ks_default_plan", "ks_hmul", "ks_hrot", "ks_eval_workspace_bytes",
            "ks_ntt", "ks_intt", "ks_bconv", "ks_modup", "ks_keymult", "ks_moddown", "ks_keyswitch",
            "ks_launch_count", "ks_strerror", "ks_last_hip_error", "ks_trace_begin", "ks_trace_end",
            "ks_graph_create", "ks_graph_launch", "ks_graph_destroy", "ks_modmul_rate", "ks_modmul_chains", "ks_copy_rate",
            "ks_keyswitch_noalloc"]


class KsError(RuntimeError):
    def __init__(self, code, what):
        msg = _lib.ks_strerror(code).decode()
        if code == KS_EHIP:
            msg += f" ({_lib.ks_last_hip_error().decode()})"
        super().__init__(f"{what}: {msg} [{code}]")
        self.code = code


def _check(rc, what):
    if rc != KS_OK:
        raise KsError(rc, what)


def _need(t, words, what):
    """Raise ValueError unless t is an int64 tensor of at least `words`
    elements: the C ABI cannot see buffer sizes, so a short buffer would be
    read or written past its end on the device."""
    if t is None:
        raise ValueError(f"{what}: missing tensor")
    if t.dtype != torch.int64:
        raise ValueError(f"{what}: expected dtype int64 (uint64 residues), got {t.dtype}")
    if words > 0 and t.numel() < words:
        raise ValueError(f"{what}: {t.numel()} elements, the call needs {words}")


def _need_bytes(t, nbytes, what):
    _need(t, 0, what)
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what}: {t.numel() * t.element_size()} bytes, the call needs {nbytes}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_plan(dataflow=DPOB, chunks=1, log_r=-1, mfma=False, split=False, tile=0, hoist=False):
    """A plan; log_r < 0 selects the library's default NTT split; mfma selects
    the int8 matrix-core BConv; split runs the two halves of a batch on two
    streams; tile > 0 runs the batch in passes of at most `tile` items; hoist
    (DPOB only) runs the raised digits' forward block pass as its own launch."""
    flags = (PLAN_MFMA_BCONV if mfma else 0) | (PLAN_SPLIT_STREAMS if split else 0) | (PLAN_HOIST_FWD if hoist else 0)
    return Plan(dataflow, chunks, log_r, flags, tile)


class KsParams:
    """Handle of one (dnum, N = 2^log_n, ell) parameter set on the current
    device, or of one of its levels (at_level)."""

    def __init__(self, dnum: int, log_n: int, ell: int, _handle=None):
        h = _vp()
        if _handle is None:
            _check(_lib.ks_params_create(dnum, log_n, ell, ctypes.byref(h)), "ks_params_create")
        else:
            h = _handle
        self._h = h
        info = Info()
        _check(_lib.ks_params_info(h, ctypes.byref(info)), "ks_params_info")
        self.n, self.log_n, self.ell, self.k = info.n, info.log_n, info.ell, info.k
        self.alpha, self.dnum, self.ndig = info.alpha, info.dnum, info.ndig
        self.key_ell = info.key_ell
        self.nl = self.ell + self.k
        self.moduli = [int(info.moduli[t]) for t in range(self.nl)]
        self.psi = [int(info.psi[t]) for t in range(self.nl)]

    def at_level(self, level: int) -> "KsParams":
        """The same set at `level` Q limbs, KeySwitched with this set's
        evaluation key (ks_params_at_level)."""
        h = _vp()
        _check(_lib.ks_params_at_level(self._h, level, ctypes.byref(h)), "ks_params_at_level")
        return KsParams(self.dnum, self.log_n, level, _handle=h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ks_params_destroy(h)
            self._h = None

    def __repr__(self):
        lv = f", level of ell={self.key_ell}" if self.key_ell != self.ell else ""
        return f"KsParams(dnum={self.dnum}, N=2^{self.log_n}, ell={self.ell}{lv}, k={self.k})"

    # ------------------------------------------------------------ queries
    def default_plan(self, batch: int = 1) -> Plan:
        p = Plan()
        _check(_lib.ks_default_plan(self._h, batch, ctypes.byref(p)), "ks_default_plan")
        return p

    def workspace_bytes(self, batch: int, plan: Plan = None) -> int:
        b = _sz()
        _check(_lib.ks_workspace_bytes(self._h, batch, ctypes.byref(plan) if plan else None, ctypes.byref(b)),
               "ks_workspace_bytes")
        return int(b.value)

    def workspace(self, batch: int, plan: Plan = None, device="cuda") -> torch.Tensor:
        nbytes = max(self.workspace_bytes(batch, plan), 8)
        return torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=device)

    def launch_count(self, batch: int, plan: Plan = None) -> int:
        rc = _lib.ks_launch_count(self._h, batch, ctypes.byref(plan) if plan else None)
        if rc < 0:
            raise KsError(rc, "ks_launch_count")
        return rc

    # ---------------------------------------------- buffer-size checks
    def _digit_size(self, j: int) -> int:
        return min((j + 1) * self.alpha, self.ell) - j * self.alpha

    def _key_words(self) -> int:
        nd, two, rows, n = self.shapes(0)["evk"]
        return nd * two * rows * n

    def _staged_ws_bytes(self, batch: int) -> int:
        return self.workspace_bytes(batch, make_plan(STAGED))

    def check_keyswitch_args(self, d, evk, out, batch, ws, plan=None, eval_ws=False, d_words=None):
        """ValueError unless every buffer of a KeySwitch-shaped call is int64
        and large enough for `batch` items (d: batch*ell*N words, or d_words;
        evk: the top-level key; out: batch*2*ell*N; ws: the workspace of the
        plan)."""
        if batch <= 0:
            return
        n, ell = self.n, self.ell
        _need(d, batch * ell * n if d_words is None else d_words, "d")
        _need(evk, self._key_words(), "evk")
        _need(out, batch * 2 * ell * n, "out")
        need = self.eval_workspace_bytes(batch, plan) if eval_ws else self.workspace_bytes(batch, plan)
        _need_bytes(ws, need, "ws")

    # -------------------------------------------------------------- calls
    def ntt(self, x, basis_first=0, n_limbs=None, batch=None, stream=None):
        n_limbs = x.shape[-2] if n_limbs is None else n_limbs
        batch = (x.numel() // (n_limbs * self.n)) if batch is None else batch
        _need(x, batch * n_limbs * self.n, "x")
        _check(_lib.ks_ntt(self._h, _ptr(x), basis_first, n_limbs, batch, _stream(stream)), "ks_ntt")

    def intt(self, x, basis_first=0, n_limbs=None, batch=None, stream=None):
        n_limbs = x.shape[-2] if n_limbs is None else n_limbs
        batch = (x.numel() // (n_limbs * self.n)) if batch is None else batch
        _need(x, batch * n_limbs * self.n, "x")
        _check(_lib.ks_intt(self._h, _ptr(x), basis_first, n_limbs, batch, _stream(stream)), "ks_intt")

    def bconv(self, src, src_set, dst, batch, stream=None):
        if batch > 0 and (src_set == KS_SET_P or 0 <= src_set < self.ndig):
            ns = self.k if src_set == KS_SET_P else self._digit_size(src_set)
            nd = self.ell if src_set == KS_SET_P else self.nl - ns
            _need(src, batch * ns * self.n, "src")
            _need(dst, batch * nd * self.n, "dst")
        _check(_lib.ks_bconv(self._h, _ptr(src), src_set, _ptr(dst), batch, _stream(stream)), "ks_bconv")

    def modup(self, d, ext, batch, ws, stream=None):
        if batch > 0:
            _need(d, batch * self.ell * self.n, "d")
            _need(ext, batch * self.ndig * self.nl * self.n, "ext")
            _need_bytes(ws, self._staged_ws_bytes(batch), "ws")
        _check(_lib.ks_modup(self._h, _ptr(d), _ptr(ext), batch, _ptr(ws), _stream(stream)), "ks_modup")

    def keymult(self, ext, evk, acc, batch, stream=None):
        if batch > 0:
            _need(ext, batch * self.ndig * self.nl * self.n, "ext")
            _need(evk, self._key_words(), "evk")
            _need(acc, batch * 2 * self.nl * self.n, "acc")
        _check(_lib.ks_keymult(self._h, _ptr(ext), _ptr(evk), _ptr(acc), batch, _stream(stream)), "ks_keymult")

    def moddown(self, acc, out, batch, ws, stream=None):
        if batch > 0:
            _need(acc, batch * 2 * self.nl * self.n, "acc")
            _need(out, batch * 2 * self.ell * self.n, "out")
            _need_bytes(ws, self._staged_ws_bytes(batch), "ws")
        _check(_lib.ks_moddown(self._h, _ptr(acc), _ptr(out), batch, _ptr(ws), _stream(stream)), "ks_moddown")

    def keyswitch(self, d, evk, out, batch, ws, plan: Plan = None, stream=None):
        self.check_keyswitch_args(d, evk, out, batch, ws, plan)
        _check(_lib.ks_keyswitch(self._h, _ptr(d), _ptr(evk), _ptr(out), batch,
                                 ctypes.byref(plan) if plan else None, _ptr(ws), _stream(stream)), "ks_keyswitch")

    def keyswitch_noalloc(self, d, evk, out, batch, plan: Plan = None, stream=None):
        """ks_keyswitch with the library's static scratch as workspace (no
        allocation); calls that overlap on one GPU race."""
        if batch > 0:
            _need(d, batch * self.ell * self.n, "d")
            _need(evk, self._key_words(), "evk")
            _need(out, batch * 2 * self.ell * self.n, "out")
        _check(_lib.ks_keyswitch_noalloc(self._h, _ptr(d), _ptr(evk), _ptr(out), batch,
                                         ctypes.byref(plan) if plan else None, _stream(stream)), "ks_keyswitch_noalloc")

    def eval_workspace_bytes(self, batch: int, plan: Plan = None) -> int:
        b = _sz()
        _check(_lib.ks_eval_workspace_bytes(self._h, batch, ctypes.byref(plan) if plan else None, ctypes.byref(b)),
               "ks_eval_workspace_bytes")
        return int(b.value)

    def eval_workspace(self, batch: int, plan: Plan = None, device="cuda") -> torch.Tensor:
        nbytes = max(self.eval_workspace_bytes(batch, plan), 8)
        return torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=device)

    def hmul(self, a, b, evk, out, batch, ws, plan: Plan = None, stream=None):
        """(a0 b0, a0 b1 + a1 b0) + KeySwitch(a1 b1); evk from s*s to s."""
        self.check_keyswitch_args(a, evk, out, batch, ws, plan, eval_ws=True, d_words=batch * 2 * self.ell * self.n)
        if batch > 0:
            _need(b, batch * 2 * self.ell * self.n, "b")
        _check(_lib.ks_hmul(self._h, _ptr(a), _ptr(b), _ptr(evk), _ptr(out), batch,
                            ctypes.byref(plan) if plan else None, _ptr(ws), _stream(stream)), "ks_hmul")

    def hrot(self, ct, galois, evk, out, batch, ws, plan: Plan = None, stream=None):
        """(sigma(c0), 0) + KeySwitch(sigma(c1)) for x -> x^galois; evk from sigma(s) to s."""
        self.check_keyswitch_args(ct, evk, out, batch, ws, plan, eval_ws=True, d_words=batch * 2 * self.ell * self.n)
        _check(_lib.ks_hrot(self._h, _ptr(ct), galois, _ptr(evk), _ptr(out), batch,
                            ctypes.byref(plan) if plan else None, _ptr(ws), _stream(stream)), "ks_hrot")

    def modmul_rate(self, kind: int, blocks: int = 4096, iters: int = 2048, reps: int = 3) -> float:
        """Measured modular products per second of one kind (0 FP64, 1 Shoup,
        2 Montgomery; ks_modmul_rate), the best of `reps` timed launches."""
        sink = torch.empty(blocks * 256, dtype=torch.int64, device="cuda")
        stream = torch.cuda.current_stream()
        ev = HipEvents(2)
        _check(_lib.ks_modmul_rate(self._h, kind, blocks, iters, _ptr(sink), _stream(stream)), "ks_modmul_rate")
        best = float("inf")
        for _ in range(reps):
            ev.record(0, stream)
            _check(_lib.ks_modmul_rate(self._h, kind, blocks, iters, _ptr(sink), _stream(stream)), "ks_modmul_rate")
            ev.record(1, stream)
            torch.cuda.synchronize()
            best = min(best, ev.elapsed_ms(0, 1))
        return blocks * 256 * _lib.ks_modmul_chains() * iters / (best / 1e3)

    def graph(self, d, evk, out, batch, ws, plan: Plan = None, stream=None) -> "Graph":
        """Capture one KeySwitch on these buffers into a replayable HIP graph."""
        return Graph(self, d, evk, out, batch, ws, plan, stream)

    # ------------------------------------------------------------ helpers
    def shapes(self, batch: int):
        n, ell, nl, nd = self.n, self.ell, self.nl, self.ndig
        key_nd = -(-self.key_ell // self.alpha)
        return {"d": (batch, ell, n), "ext": (batch, nd, nl, n), "evk": (key_nd, 2, self.key_ell + self.k, n),
                "acc": (batch, 2, nl, n), "out": (batch, 2, ell, n)}


def copy_rate(kind: int, nt: bool, words: int = 1 << 27, blocks: int = 4096, reps: int = 3) -> float:
    """Measured HBM bytes per second (read + write) of the library's copy
    probe over `words` words (ks_copy_rate), the best of `reps` launches."""
    src = torch.ones(words, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    ev = HipEvents(2)
    args = (kind, int(nt), blocks, _ptr(src), _ptr(dst), words, _stream(stream))
    _check(_lib.ks_copy_rate(*args), "ks_copy_rate")
    best = float("inf")
    for _ in range(reps):
        ev.record(0, stream)
        _check(_lib.ks_copy_rate(*args), "ks_copy_rate")
        ev.record(1, stream)
        torch.cuda.synchronize()
        best = min(best, ev.elapsed_ms(0, 1))
    return 16 * words / (best / 1e3)


class Graph:
    """A captured KeySwitch (ks_graph_*); keeps its buffers alive while it lives."""

    def __init__(self, params, d, evk, out, batch, ws, plan=None, stream=None):
        params.check_keyswitch_args(d, evk, out, batch, ws, plan)
        if stream is None:
            stream = torch.cuda.current_stream()
        if stream.cuda_stream == 0:
            raise ValueError("graph capture needs a non-default stream")
        h = _vp()
        _check(_lib.ks_graph_create(params._h, _ptr(d), _ptr(evk), _ptr(out), batch,
                                    ctypes.byref(plan) if plan else None, _ptr(ws), _stream(stream), ctypes.byref(h)),
               "ks_graph_create")
        self._h = h
        self._keep = (params, d, evk, out, ws, plan)

    def launch(self, stream=None):
        _check(_lib.ks_graph_launch(self._h, _stream(stream)), "ks_graph_launch")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ks_graph_destroy(h)
            self._h = None


class HipEvents:
    """A pool of HIP timing events, created through the HIP runtime."""

    _hip = None

    @staticmethod
    def runtime():
        if HipEvents._hip is None:
            h = ctypes.CDLL("libamdhip64.so")
            h.hipEventCreate.argtypes = [ctypes.POINTER(_vp)]
            h.hipEventDestroy.argtypes = [_vp]
            h.hipEventRecord.argtypes = [_vp, _vp]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), _vp, _vp]
            HipEvents._hip = h
        return HipEvents._hip

    def __init__(self, count: int):
        h = HipEvents.runtime()
        self.ev = (_vp * count)()
        self.count = 0
        for i in range(count):
            e = _vp()
            rc = h.hipEventCreate(ctypes.byref(e))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed ({rc})")
            self.ev[i] = e.value
            self.count = i + 1

    def record(self, i: int, stream=None) -> None:
        rc = HipEvents._hip.hipEventRecord(self.ev[i], _stream(stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_ms(self, i: int, j: int) -> float:
        ms = ctypes.c_float()
        rc = HipEvents._hip.hipEventElapsedTime(ctypes.byref(ms), self.ev[i], self.ev[j])
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def __del__(self):
        try:
            h = HipEvents._hip
            for i in range(getattr(self, "count", 0)):
                h.hipEventDestroy(self.ev[i])
        except Exception:  # interpreter shutdown: the runtime may be gone
            pass


def trace_begin(events: HipEvents, kind_mask: int = 0xFFFFFFFF) -> None:
    """Bracket the following kernel launches of the chosen kinds with events[2i], events[2i+1]."""
    _check(_lib.ks_trace_begin(ctypes.cast(events.ev, ctypes.POINTER(_vp)), events.count // 2, kind_mask),
           "ks_trace_begin")


def trace_end(capacity: int = 4096):
    """Stop tracing; returns the kind of every recorded launch, in order."""
    kinds = (_i * capacity)()
    n = _lib.ks_trace_end(kinds, capacity)
    return [int(kinds[i]) for i in range(min(n, capacity))]


def raw_call(name, *args):
    """Direct access to an exported symbol (tests of the argument checks)."""
    return getattr(_lib, name)(*args)
