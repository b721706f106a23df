"""Reduced-history Feynman amplitudes on one AMD MI355X (gfx950).

Thin ctypes binding over the C ABI in include/fhs.h: argument marshalling
only.  Every step of the computation runs in the native library
(libfhs.so: host reducer + HIP kernels); PyTorch provides device memory and
streams.  There is no CPU fallback: if the library is missing, importing the
native handle raises.

    prog = Program(circuit_text)            # fhs_reduce (host)
    ctx = Context(device=0)
    ctx.load(prog)                          # fhs_load_program
    ctx.set_partition(*prog.choose_partition(PART_EQ8))
    amps, stats = ctx.evaluate(inputs, coeffs, outputs, threshold=0.0)
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfhs.so")

PART_NONE, PART_THIRDS, PART_EQ8, PART_MODEL = 0, 1, 2, 3
REDUCE_FUSE = 1
REDUCE_PAIR = 2
REDUCE_FORWARD = 4
REDUCE_OPTIMAL = 8
REDUCE_GREEDY = 16
PLACEMENTS = {"backward": 0, "forward": REDUCE_FORWARD, "optimal": REDUCE_OPTIMAL, "greedy": REDUCE_GREEDY}

STATUS = {0: "FHS_OK", 1: "FHS_EINVAL", 2: "FHS_EUNSUPPORTED", 3: "FHS_ERANGE",
          4: "FHS_ENOMEM", 5: "FHS_EHIP", 6: "FHS_ESTATE", 7: "FHS_EPARSE"}

EXPORTS = [
    "fhs_status_string", "fhs_reduce", "fhs_reduce_ex", "fhs_program_free", "fhs_program_get_info",
    "fhs_program_sources", "fhs_partition_cost", "fhs_choose_partition", "fhs_ctx_create",
    "fhs_ctx_destroy", "fhs_last_error", "fhs_load_program", "fhs_set_partition",
    "fhs_get_partition", "fhs_set_table_budget", "fhs_workspace_size", "fhs_evaluate",
    "fhs_evaluate_plain", "fhs_set_launch_config", "fhs_get_launch_config",
    "fhs_program_work", "fhs_set_kernel_timing", "fhs_kernel_times", "fhs_kernel_counts", "fhs_get_plan",
    "fhs_split_features", "fhs_candidate_splits", "fhs_cut_allowed", "fhs_load_cost_model",
    "fhs_precompile", "fhs_choose_partition_ctx", "fhs_predict_splits", "fhs_mlp_param_count", "fhs_mlp_workspace_size",
    "fhs_mlp_forward", "fhs_mlp_backward", "fhs_mlp_adam", "fhs_evaluate_noalloc",
    "fhs_item_stamps",
]

NOALLOC_SCRATCH_BYTES = 256 << 20   # FHS_NOALLOC_SCRATCH_BYTES

N_FEATURES = 16


class FhsError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}" if msg else STATUS.get(status, str(status)))


class ProgramInfo(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_uint32), ("n_gates", ctypes.c_uint32),
                ("n_sources", ctypes.c_uint32), ("n_words", ctypes.c_uint32),
                ("n_leading", ctypes.c_uint32), ("n_branch", ctypes.c_uint32),
                ("forward", ctypes.c_uint32)]


class Work(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_uint64), ("int_ops", ctypes.c_uint64),
                ("fp64_flops", ctypes.c_uint64), ("branch", ctypes.c_uint64),
                ("src_int_ops", ctypes.c_uint64), ("hoist_int_ops", ctypes.c_uint64),
                ("hoist_fp64_flops", ctypes.c_uint64), ("count_int_ops", ctypes.c_uint64),
                ("count_fp64_flops", ctypes.c_uint64), ("hoist_count_int_ops", ctypes.c_uint64),
                ("hoist_count_fp64_flops", ctypes.c_uint64)]


class Plan(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in (
        "c1", "c2", "Ap", "Ar", "As", "n_batches", "pairs_per_batch", "chunk", "items_per_pair",
        "lanes_per_root_task", "plain_blocks_per_pair")] + [("table_bytes", ctypes.c_uint64)] + [
        ("prefix_depth_first", ctypes.c_uint32), ("items_per_claim", ctypes.c_uint32),
        ("count_groups", ctypes.c_uint32), ("count_entries", ctypes.c_uint32),
        ("root_parts", ctypes.c_uint32), ("pair_filter", ctypes.c_uint32)]


class MlpShape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_uint32), ("h1", ctypes.c_uint32), ("h2", ctypes.c_uint32)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("histories_per_lane", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("dispatch", ctypes.c_uint32),
                ("items_per_claim", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The native library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2608_01467_amd._build`")
        L = ctypes.CDLL(LIB_PATH)
        P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        pU32 = ctypes.POINTER(U32)
        L.fhs_status_string.restype = ctypes.c_char_p
        L.fhs_status_string.argtypes = [I32]
        L.fhs_reduce.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(P)]
        L.fhs_reduce_ex.argtypes = [ctypes.c_char_p, ctypes.c_size_t, U32, ctypes.POINTER(P)]
        L.fhs_program_free.argtypes = [P]
        L.fhs_program_free.restype = None
        L.fhs_program_get_info.argtypes = [P, ctypes.POINTER(ProgramInfo)]
        L.fhs_program_sources.argtypes = [P, pU32, U32]
        L.fhs_partition_cost.argtypes = [P, U32, U32, ctypes.POINTER(U64), pU32]
        L.fhs_choose_partition.argtypes = [P, I32, pU32, pU32]
        L.fhs_ctx_create.argtypes = [I32, ctypes.POINTER(P)]
        L.fhs_ctx_destroy.argtypes = [P]
        L.fhs_ctx_destroy.restype = None
        L.fhs_last_error.argtypes = [P]
        L.fhs_last_error.restype = ctypes.c_char_p
        L.fhs_load_program.argtypes = [P, P]
        L.fhs_set_partition.argtypes = [P, U32, U32]
        L.fhs_get_partition.argtypes = [P, pU32, pU32]
        L.fhs_set_table_budget.argtypes = [P, ctypes.c_size_t]
        L.fhs_workspace_size.argtypes = [P, U32, U32, ctypes.POINTER(ctypes.c_size_t)]
        L.fhs_program_work.argtypes = [P, U32, U32, ctypes.POINTER(Work)]
        L.fhs_set_kernel_timing.argtypes = [P, I32]
        L.fhs_get_plan.argtypes = [P, U32, U32, ctypes.POINTER(Plan)]
        L.fhs_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_float), U32, ctypes.POINTER(U32)]
        L.fhs_kernel_counts.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.fhs_item_stamps.argtypes = [P, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), pU32,
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.fhs_set_launch_config.argtypes = [P, ctypes.POINTER(LaunchConfig)]
        pD = ctypes.POINTER(ctypes.c_double)
        L.fhs_split_features.argtypes = [P, U32, U32, U32, U32, pD]
        L.fhs_candidate_splits.argtypes = [P, pU32, pU32, U32, pU32]
        L.fhs_cut_allowed.argtypes = [P, U32, ctypes.POINTER(ctypes.c_int)]
        L.fhs_load_cost_model.argtypes = [P, pD, ctypes.c_size_t]
        L.fhs_choose_partition_ctx.argtypes = [P, I32, U32, U32, pU32, pU32]
        L.fhs_predict_splits.argtypes = [P, U32, U32, pU32, pU32, U32, pD]
        L.fhs_precompile.argtypes = [P, pU32, pU32, U32, U32, U32, ctypes.c_double, U32, pU32]
        pS = ctypes.POINTER(MlpShape)
        L.fhs_mlp_param_count.argtypes = [pS, ctypes.POINTER(ctypes.c_size_t)]
        L.fhs_mlp_workspace_size.argtypes = [pS, U32, ctypes.POINTER(ctypes.c_size_t)]
        L.fhs_mlp_forward.argtypes = [pS, P, P, U32, P, P, P]
        L.fhs_mlp_backward.argtypes = [pS, P, P, P, U32, P, P, P, ctypes.c_size_t, P]
        L.fhs_mlp_adam.argtypes = [ctypes.c_size_t, P, P, P, P, U32, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.fhs_get_launch_config.argtypes = [P, ctypes.POINTER(LaunchConfig)]
        ev = [P, P, P, U32, P, U32, ctypes.c_double, P, P, P, ctypes.c_size_t, P]
        L.fhs_evaluate.argtypes = ev
        L.fhs_evaluate_plain.argtypes = ev
        L.fhs_evaluate_noalloc.argtypes = [P, P, P, U32, P, U32, ctypes.c_double, P, P, P]
        _lib = L
    return _lib


def _check(st: int, ctx=None) -> None:
    if st != 0:
        msg = ""
        if ctx is not None and ctx._h:
            msg = lib().fhs_last_error(ctx._h).decode()
        raise FhsError(st, msg)


class Program:
    """Host-side reduced-history program (fhs_reduce)."""

    def __init__(self, circuit_text: str, fuse: bool = True, pair: bool = True,
                 forward: bool = False, placement: str = "backward"):
        """fuse: fold add/subtract ladders (FHS_REDUCE_FUSE); pair: also merge
        complementary folded ladders (FHS_REDUCE_PAIR, only with fuse);
        placement: "backward" (the sweep from the output), "forward" (the
        sweep from the input, FHS_REDUCE_FORWARD; positions and cuts then
        count from the input), "optimal" or "greedy" (by determinism
        reachability, FHS_REDUCE_OPTIMAL / FHS_REDUCE_GREEDY); forward=True
        is placement="forward"."""
        if placement not in PLACEMENTS:
            raise ValueError(f"placement must be one of {sorted(PLACEMENTS)}")
        if forward:
            placement = "forward"
        b = circuit_text.encode()
        h = ctypes.c_void_p()
        flags = (REDUCE_FUSE | (REDUCE_PAIR if pair else 0)) if fuse else 0
        flags |= PLACEMENTS[placement]
        self.placement = placement
        _check(lib().fhs_reduce_ex(b, len(b), flags, ctypes.byref(h)))
        self._h = h
        info = ProgramInfo()
        _check(lib().fhs_program_get_info(h, ctypes.byref(info)))
        self.n = info.n_qubits
        self.G = info.n_gates
        self.A = info.n_sources
        self.W = info.n_words
        self.L = info.n_leading
        self.n_branch = info.n_branch
        self.forward = bool(info.forward)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fhs_program_free(self._h)
            self._h = None

    @property
    def source_eval_positions(self) -> list:
        arr = (ctypes.c_uint32 * max(1, self.A))()
        _check(lib().fhs_program_sources(self._h, arr, self.A))
        return list(arr[: self.A])

    def partition_cost(self, c1: int, c2: int) -> Tuple[int, Tuple[int, ...]]:
        cost = (ctypes.c_uint64 * 2)()
        reg = (ctypes.c_uint32 * 6)()
        _check(lib().fhs_partition_cost(self._h, c1, c2, cost, reg))
        return int(cost[0]) | (int(cost[1]) << 64), tuple(reg)

    def work(self, e0: int, e1: int) -> dict:
        """Algorithmic work of evaluation positions [e0, e1) per history."""
        w = Work()
        _check(lib().fhs_program_work(self._h, e0, e1, ctypes.byref(w)))
        return {k: getattr(w, k) for k, _ in Work._fields_}

    def split_features(self, c1: int, c2: int, M: int, S: int) -> np.ndarray:
        out = (ctypes.c_double * N_FEATURES)()
        _check(lib().fhs_split_features(self._h, c1, c2, M, S, out))
        return np.array(out[:], dtype=np.float64)

    def candidate_splits(self) -> list:
        n = ctypes.c_uint32()
        _check(lib().fhs_candidate_splits(self._h, None, None, 0, ctypes.byref(n)))
        a = (ctypes.c_uint32 * max(1, n.value))()
        b = (ctypes.c_uint32 * max(1, n.value))()
        _check(lib().fhs_candidate_splits(self._h, a, b, n.value, ctypes.byref(n)))
        return list(zip(a[: n.value], b[: n.value]))

    def cut_allowed(self, c: int) -> bool:
        """Whether a cut may fall at evaluation position c (fhs_cut_allowed)."""
        ok = ctypes.c_int()
        _check(lib().fhs_cut_allowed(self._h, c, ctypes.byref(ok)))
        return bool(ok.value)

    def choose_partition(self, mode: int = PART_EQ8) -> Tuple[int, int]:
        c1, c2 = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().fhs_choose_partition(self._h, mode, ctypes.byref(c1), ctypes.byref(c2)))
        return c1.value, c2.value


def _to_words(values, n: int) -> np.ndarray:
    w = max(1, (n + 63) // 64)
    if isinstance(values, np.ndarray) and values.dtype == np.uint64:
        arr = np.ascontiguousarray(values.reshape(-1, w))
    else:
        arr = np.zeros((len(values), w), dtype=np.uint64)
        for i, v in enumerate(values):
            v = int(v)
            if v < 0 or v >> n:
                raise ValueError(f"bitstring {v:#x} has bits at or above n={n}")
            for j in range(w):
                arr[i, j] = (v >> (64 * j)) & ((1 << 64) - 1)
    return arr


class Context:
    """One device, one loaded program (fhs_ctx)."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = device
        h = ctypes.c_void_p()
        st = lib().fhs_ctx_create(device, ctypes.byref(h))
        if st != 0:
            raise FhsError(st, f"cannot create a context on HIP device {device}")
        self._h = h
        self._ws = None
        self.program: Optional[Program] = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fhs_ctx_destroy(self._h)
            self._h = None

    def load(self, prog: Program) -> None:
        _check(lib().fhs_load_program(self._h, prog._h), self)
        self.program = prog

    def set_partition(self, c1: int, c2: int) -> None:
        _check(lib().fhs_set_partition(self._h, c1, c2), self)

    @property
    def partition(self) -> Tuple[int, int]:
        c1, c2 = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().fhs_get_partition(self._h, ctypes.byref(c1), ctypes.byref(c2)), self)
        return c1.value, c2.value

    def set_launch_config(self, histories_per_lane: int = 0, chunk: int = 0,
                          blocks_per_cu: int = 0, dispatch: int = 0, items_per_claim: int = 0) -> None:
        cfg = LaunchConfig(histories_per_lane, chunk, blocks_per_cu, dispatch, items_per_claim)
        _check(lib().fhs_set_launch_config(self._h, ctypes.byref(cfg)), self)

    def precompile(self, splits, M: int, S: int, threshold: float = 0.0, threads: int = 16) -> int:
        """Compile the dispatch-mode-3 consumers for these splits ahead of
        time in up to `threads` helper processes (fhs_precompile); returns
        how many were compiled (0 in the other dispatch modes)."""
        splits = list(splits)
        n = len(splits)
        a = (ctypes.c_uint32 * max(n, 1))(*[int(c[0]) for c in splits])
        b = (ctypes.c_uint32 * max(n, 1))(*[int(c[1]) for c in splits])
        done = ctypes.c_uint32(0)
        _check(lib().fhs_precompile(self._h, a, b, n, M, S, float(threshold), threads,
                                    ctypes.byref(done)), self)
        return done.value

    @property
    def launch_config(self) -> Tuple[int, int, int, int]:
        cfg = LaunchConfig()
        _check(lib().fhs_get_launch_config(self._h, ctypes.byref(cfg)), self)
        return cfg.histories_per_lane, cfg.chunk, cfg.blocks_per_cu, cfg.dispatch

    @property
    def items_per_claim(self) -> int:
        """The launch configuration's items per claim (0: automatic)."""
        cfg = LaunchConfig()
        _check(lib().fhs_get_launch_config(self._h, ctypes.byref(cfg)), self)
        return cfg.items_per_claim

    def plan(self, M: int, S: int) -> dict:
        p = Plan()
        _check(lib().fhs_get_plan(self._h, M, S, ctypes.byref(p)), self)
        return {k: getattr(p, k) for k, _ in Plan._fields_}

    def load_cost_model(self, blob) -> None:
        arr = np.ascontiguousarray(np.asarray(blob, dtype=np.float64))
        _check(lib().fhs_load_cost_model(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         arr.size), self)

    def choose_partition(self, mode: int, M: int, S: int = 1) -> Tuple[int, int]:
        c1, c2 = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().fhs_choose_partition_ctx(self._h, mode, M, S, ctypes.byref(c1),
                                              ctypes.byref(c2)), self)
        return c1.value, c2.value

    def predict_splits(self, splits, M: int, S: int = 1) -> np.ndarray:
        """Predicted log(seconds) per split (NaN outside the training range)."""
        n = len(splits)
        a = (ctypes.c_uint32 * max(1, n))(*[c[0] for c in splits])
        b = (ctypes.c_uint32 * max(1, n))(*[c[1] for c in splits])
        out = (ctypes.c_double * max(1, n))()
        _check(lib().fhs_predict_splits(self._h, M, S, a, b, n, out), self)
        return np.array(out[:n], dtype=np.float64)

    def set_kernel_timing(self, enable: bool) -> None:
        _check(lib().fhs_set_kernel_timing(self._h, 1 if enable else 0), self)

    def kernel_counts(self) -> Tuple[int, int]:
        """(prefix entries built, prefix entries still consistent) of the last
        evaluation in timing mode."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().fhs_kernel_counts(self._h, ctypes.byref(a), ctypes.byref(b)), self)
        return a.value, b.value

    def item_stamps(self):
        """(stamps uint64 [items, 2] start/end, items per pair, clock ticks
        per second) of the last batched evaluation in timing mode."""
        n = ctypes.c_size_t()
        ipp = ctypes.c_uint32()
        tps = ctypes.c_uint64()
        _check(lib().fhs_item_stamps(self._h, None, 0, ctypes.byref(n), ctypes.byref(ipp),
                                     ctypes.byref(tps)), self)
        arr = np.zeros((n.value, 2), dtype=np.uint64)
        _check(lib().fhs_item_stamps(self._h, arr.ctypes.data, n.value, ctypes.byref(n),
                                     ctypes.byref(ipp), ctypes.byref(tps)), self)
        return arr, ipp.value, tps.value

    def kernel_times(self) -> list:
        """Durations (ms) of the hot-kernel launches of the last evaluation."""
        n = ctypes.c_uint32()
        buf = (ctypes.c_float * 4096)()
        _check(lib().fhs_kernel_times(self._h, buf, 4096, ctypes.byref(n)), self)
        return [float(buf[i]) for i in range(min(n.value, 4096))]

    def set_table_budget(self, nbytes: int) -> None:
        _check(lib().fhs_set_table_budget(self._h, nbytes), self)

    def workspace_size(self, M: int, S: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().fhs_workspace_size(self._h, M, S, ctypes.byref(b)), self)
        return b.value

    def workspace(self, nbytes: int):
        torch = self._torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def device_bits(self, values):
        """Bitstrings (ints or uint64 words) -> int64 device tensor [count, W]."""
        torch = self._torch
        if isinstance(values, torch.Tensor):
            return values.contiguous()
        arr = _to_words(values, self.program.n)
        return torch.from_numpy(arr.view(np.int64)).to(f"cuda:{self.device}")

    def device_coeffs(self, coeffs):
        torch = self._torch
        if isinstance(coeffs, torch.Tensor):
            return coeffs.contiguous()
        arr = np.zeros((len(coeffs), 2), dtype=np.float64)
        for i, z in enumerate(coeffs):
            z = complex(*z) if isinstance(z, tuple) else complex(z)
            arr[i] = (z.real, z.imag)
        return torch.from_numpy(arr).to(f"cuda:{self.device}")

    def evaluate(self, inputs, coeffs, outputs, threshold: float = 0.0, plain: bool = False,
                 out=None, stream=None):
        """<b_out|C|psi> for each output.  Returns (amps float64 [M,2],
        stats int64 [M,4]) on the device; results are complete once the
        stream (default: torch's current stream) has synchronized."""
        torch = self._torch
        d_in = self.device_bits(inputs)
        d_out = self.device_bits(outputs)
        d_cf = self.device_coeffs(coeffs)
        S, M = d_in.shape[0], d_out.shape[0]
        if out is None:
            amps = torch.empty((M, 2), dtype=torch.float64, device=d_out.device)
            stats = torch.empty((M, 4), dtype=torch.int64, device=d_out.device)
        else:
            amps, stats = out
        nbytes = self.workspace_size(M, max(S, 1))
        ws = self.workspace(nbytes)
        if stream is None:
            stream = torch.cuda.current_stream(d_out.device).cuda_stream
        fn = lib().fhs_evaluate_plain if plain else lib().fhs_evaluate
        _check(fn(self._h, d_in.data_ptr(), d_cf.data_ptr(), S, d_out.data_ptr(), M,
                  float(threshold), amps.data_ptr(), stats.data_ptr(), ws.data_ptr(),
                  ws.numel(), ctypes.c_void_p(stream)), self)
        return amps, stats

    def evaluate_noalloc(self, inputs, coeffs, outputs, threshold: float = 0.0, out=None,
                         stream=None):
        """As evaluate(), through fhs_evaluate_noalloc: the library's static
        scratch instead of a workspace, nothing allocated by the call (the
        argument tensors are created here when not given as device tensors)."""
        torch = self._torch
        d_in = self.device_bits(inputs)
        d_out = self.device_bits(outputs)
        d_cf = self.device_coeffs(coeffs)
        S, M = d_in.shape[0], d_out.shape[0]
        if out is None:
            amps = torch.empty((M, 2), dtype=torch.float64, device=d_out.device)
            stats = torch.empty((M, 4), dtype=torch.int64, device=d_out.device)
        else:
            amps, stats = out
        if stream is None:
            stream = torch.cuda.current_stream(d_out.device).cuda_stream
        _check(lib().fhs_evaluate_noalloc(self._h, d_in.data_ptr(), d_cf.data_ptr(), S,
                                          d_out.data_ptr(), M, float(threshold), amps.data_ptr(),
                                          stats.data_ptr(), ctypes.c_void_p(stream)), self)
        return amps, stats


# ---------------------------------------------------------------------------
# Cost-model network on the device (fhs_mlp_*): thin wrappers over torch tensors
# ---------------------------------------------------------------------------

def mlp_param_count(n_in: int, h1: int, h2: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().fhs_mlp_param_count(ctypes.byref(MlpShape(n_in, h1, h2)), ctypes.byref(n)))
    return n.value


def _stream_ptr(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_forward(shape, params, x, y, act=None) -> None:
    """y[b] = network(x[b]) (device tensors, float64)."""
    sh = MlpShape(*shape)
    _check(lib().fhs_mlp_forward(ctypes.byref(sh), params.data_ptr(), x.data_ptr(), x.shape[0],
                                 y.data_ptr(), act.data_ptr() if act is not None else None,
                                 _stream_ptr(x)))


def mlp_backward(shape, params, x, t, grad, loss, ws) -> None:
    sh = MlpShape(*shape)
    _check(lib().fhs_mlp_backward(ctypes.byref(sh), params.data_ptr(), x.data_ptr(), t.data_ptr(),
                                  x.shape[0], grad.data_ptr(),
                                  loss.data_ptr() if loss is not None else None,
                                  ws.data_ptr(), ws.numel(), _stream_ptr(x)))


def mlp_workspace_size(shape, B: int) -> int:
    n = ctypes.c_size_t()
    _check(lib().fhs_mlp_workspace_size(ctypes.byref(MlpShape(*shape)), B, ctypes.byref(n)))
    return n.value


def mlp_adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    _check(lib().fhs_mlp_adam(params.numel(), params.data_ptr(), grad.data_ptr(), m.data_ptr(),
                              v.data_ptr(), step, lr, beta1, beta2, eps, _stream_ptr(params)))
