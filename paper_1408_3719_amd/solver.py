"""Python binding of the aderweno library: argument marshalling only.

Every step of the scheme runs in the HIP kernels of libaderweno.so; PyTorch
supplies the device workspace and the stream.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import _lib

MESH_VELOCITY = {"lagrangian": 0, "eulerian": 1}
FLUX = {"rusanov": 0, "osher": 1, "hll": 2}


@dataclasses.dataclass
class Config:
    M: int = 2
    gamma: float = 1.4
    cfl: float = 0.5
    levels: int = 1
    n_picard: int = 0
    mesh_velocity: str = "lagrangian"
    weno_eps: float = 1e-14
    weno_r: float = 8.0
    weno_lambda: float = 1e5
    flux: str = "rusanov"          # "rusanov", "osher" or "hll"
    lts_step_fraction: float = 0.95

    def to_c(self) -> _lib.AderConfig:
        return _lib.AderConfig(self.M, FLUX[self.flux], self.gamma, self.cfl, self.levels,
                               self.n_picard,
                               MESH_VELOCITY[self.mesh_velocity], self.weno_eps, self.weno_r,
                               self.weno_lambda, self.lts_step_fraction)


def _check(lib, ctx, code):
    if code != 0:
        msg = lib.ader_last_error(ctx).decode() if ctx else ""
        raise _lib.AderError(code, msg)


def _shape(what, M, NE, NV, NF, ne):
    nb = (M + 1) * (M + 2) // 2
    T = nG = M + 1
    return {
        "Q": (4, NE), "A": (NE,), "XE": (6, NE), "TICK": (NE,), "STEP": (NE,), "DTCFL": (NE,),
        "QM": (4, NE), "HM": (3, NE), "WNOD": (nb, 4, NE), "AVG": (T, 4, NE),
        "TRACE": (3, nG, T, 4, NE), "VVEL": (3, T, 2, NE), "X": (2, NV), "NTICK": (NV,),
        "SCAL": (4,), "TOPO_EDGES": (NF, 6), "TOPO_STENCILS": (NE, 7, ne),
        "TAB_DXI": (nb, nb), "TAB_DETA": (nb, nb), "TAB_AMEAN": (nb,), "TAB_EDGE": (3, nG, nb),
        "TAB_AT": (M, T), "TAB_BT": (M,), "TAB_DT": (T, T), "TAB_PSIC": (nb, nb),
        "TAB_SIGMA": (nb, nb), "TAB_GAUSS": (2, nG),
    }.get(what)


class _Base:
    def __init__(self, nodes, tris, bedges, cfg: Config, stream=None):
        self.lib = _lib.load()
        self.cfg = cfg
        self.ctx = ctypes.c_void_p()
        c = cfg.to_c()
        rc = self.lib.ader_create(ctypes.byref(c), ctypes.c_void_p(stream or 0), ctypes.byref(self.ctx))
        if rc != 0:
            raise _lib.AderError(rc, "ader_create rejected the configuration")
        self._nodes = np.ascontiguousarray(nodes, np.float64)
        self._tris = np.ascontiguousarray(tris, np.int32)
        be = np.zeros((0, 3), np.int32) if bedges is None else bedges
        self._bedges = np.ascontiguousarray(be, np.int32)
        self.NV, self.NE = self._nodes.shape[0], self._tris.shape[0]
        _check(self.lib, self.ctx, self.lib.ader_upload_mesh(
            self.ctx, self.NV, self._nodes.ctypes.data, self.NE, self._tris.ctypes.data,
            self._bedges.shape[0], self._bedges.ctypes.data if self._bedges.size else None))
        self.NF = self._size("TOPO_EDGES") // (6 * 4)
        self.ne = (cfg.M + 1) * (cfg.M + 2)

    def _size(self, what):
        n = ctypes.c_size_t()
        _check(self.lib, self.ctx, self.lib.ader_debug_size(self.ctx, _lib.DBG[what], ctypes.byref(n)))
        return n.value

    def dump(self, what):
        nbytes = self._size(what)
        dt = np.int32 if what in _lib.INT_ARRAYS else np.float64
        out = np.empty(nbytes // np.dtype(dt).itemsize, dt)
        _check(self.lib, self.ctx, self.lib.ader_debug_dump(self.ctx, _lib.DBG[what],
                                                            out.ctypes.data, nbytes))
        shp = _shape(what, self.cfg.M, self.NE, self.NV, self.NF, self.ne)
        return out.reshape(shp) if shp is not None else out

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ader_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostTopology(_Base):
    """Host-only view of the library's topology, stencils and tables (no GPU)."""


class Solver(_Base):
    """Moving-mesh ADER-WENO solver on one GPU.

    nodes (NV,2), tris (NE,3) CCW, bedges (NB,3) = (a, b, tag); tags 1 =
    transmissive, 2 = slip wall.  Q0 (NE,4) conserved initial averages.
    """

    def __init__(self, nodes, tris, bedges, Q0, cfg: Config, t0: float = 0.0, device="cuda:0",
                 instance_first=None):
        import torch   # loaded before the library so both share one HIP runtime
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        super().__init__(nodes, tris, bedges, cfg, stream=self.stream.cuda_stream)
        self.n_instances = 1
        if instance_first is not None:
            f = np.ascontiguousarray(instance_first, np.int32)
            self.n_instances = f.size - 1
            _check(self.lib, self.ctx, self.lib.ader_set_instances(self.ctx, self.n_instances, f.ctypes.data))
        n = ctypes.c_size_t()
        _check(self.lib, self.ctx, self.lib.ader_workspace_size(self.ctx, ctypes.byref(n)))
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        _check(self.lib, self.ctx, self.lib.ader_bind_workspace(self.ctx, ctypes.c_void_p(aligned), n.value))
        self.upload_state(Q0, t0)

    def upload_state(self, Q0, t0=0.0, X=None):
        """Q0: (NE, 4) array, or a device tensor [4][NE] (used in place); X:
        node positions (NV, 2) (array or device tensor), default the mesh's."""
        torch = self.torch
        if torch.is_tensor(Q0) and Q0.is_cuda:
            q = Q0.to(dtype=torch.float64).contiguous()
            if tuple(q.shape) != (4, self.NE):
                raise ValueError(f"a device state must be [4][{self.NE}]")
        else:
            q = torch.as_tensor(np.ascontiguousarray(np.asarray(Q0, np.float64).T), device=self.device)
            q = q.contiguous()
        x = self._devxy(X, "X") if X is not None else None
        _check(self.lib, self.ctx, self.lib.ader_upload_state_xy(
            self.ctx, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(x.data_ptr()) if x is not None else None, t0))
        self.stream.synchronize()

    def download_x(self):
        """The node positions as a device tensor (NV, 2)."""
        X = self.torch.empty((self.NV, 2), dtype=self.torch.float64, device=self.device)
        _check(self.lib, self.ctx, self.lib.ader_download_state(
            self.ctx, None, ctypes.c_void_p(X.data_ptr()), None))
        return X

    def _stats(self, st):
        return {f: getattr(st, f) for f, _ in _lib.AderStats._fields_}

    def _dev4(self, a, what):
        torch = self.torch
        if not torch.is_tensor(a):
            a = torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float64).T), device=self.device)
        a = a.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(a.shape) != (4, self.NE):
            raise ValueError(f"{what} must be [4][{self.NE}] on the device or ({self.NE}, 4)")
        return a

    def adjoint_gts_step(self, dt, qbar_next, q=None):
        """(dQ^{n+1}/dQ^n)^T qbar_next for one global step of length dt on a
        fixed mesh (dt held fixed), at the averages q (default: the current
        state).  qbar_next, q: (NE, 4) arrays or device tensors [4][NE];
        returns a device tensor [4][NE]."""
        torch = self.torch
        qn = self._dev4(qbar_next, "qbar_next")
        qs = self._dev4(q, "q") if q is not None else None
        out = torch.empty_like(qn)
        if getattr(self, "_adj_ws", None) is None:
            n = ctypes.c_size_t()
            _check(self.lib, self.ctx, self.lib.ader_adjoint_workspace_size(self.ctx, ctypes.byref(n)))
            self._adj_ws = (torch.empty(n.value + 256, dtype=torch.uint8, device=self.device), n.value)
        buf, n = self._adj_ws
        aligned = (buf.data_ptr() + 255) // 256 * 256
        _check(self.lib, self.ctx, self.lib.ader_adjoint_gts_step(
            self.ctx, dt, ctypes.c_void_p(qs.data_ptr()) if qs is not None else None,
            ctypes.c_void_p(qn.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(aligned), n))
        return out

    def adjoint_gts_step_static(self, dt, qbar_next, q=None, out=None):
        """The same step adjoint through ader_adjoint_gts_step_static: its
        scratch is the library's fixed device array, nothing is allocated by
        the library (out: optional caller tensor [4][NE] for the result)."""
        qn = self._dev4(qbar_next, "qbar_next")
        qs = self._dev4(q, "q") if q is not None else None
        if out is None:
            out = self.torch.empty_like(qn)
        _check(self.lib, self.ctx, self.lib.ader_adjoint_gts_step_static(
            self.ctx, dt, ctypes.c_void_p(qs.data_ptr()) if qs is not None else None,
            ctypes.c_void_p(qn.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def _devxy(self, a, what):
        torch = self.torch
        if not torch.is_tensor(a):
            a = torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float64)), device=self.device)
        a = a.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(a.shape) != (self.NV, 2):
            raise ValueError(f"{what} must be ({self.NV}, 2)")
        return a

    def adjoint_lagrangian_step(self, dt, qbar_next, xbar_next, q=None, x=None):
        """Adjoint of one global step of length dt on the mesh moving with the
        fluid (dt held fixed), at averages q and node positions x (default:
        the current state).  qbar_next, q: (NE, 4) arrays or device tensors
        [4][NE]; xbar_next, x: (NV, 2).  Returns device tensors (qbar [4][NE],
        xbar (NV, 2), q_next [4][NE], x_next (NV, 2)): the adjoints at the step
        start and the step's own result."""
        torch = self.torch
        qn = self._dev4(qbar_next, "qbar_next")
        xn = self._devxy(xbar_next, "xbar_next")
        qs = self._dev4(q, "q") if q is not None else None
        xs = self._devxy(x, "x") if x is not None else None
        qbar, q_next = torch.empty_like(qn), torch.empty_like(qn)
        xbar, x_next = torch.empty_like(xn), torch.empty_like(xn)
        if getattr(self, "_lag_ws", None) is None:
            n = ctypes.c_size_t()
            _check(self.lib, self.ctx, self.lib.ader_adjoint_lagrangian_workspace_size(self.ctx, ctypes.byref(n)))
            self._lag_ws = (torch.empty(n.value + 256, dtype=torch.uint8, device=self.device), n.value)
        buf, n = self._lag_ws
        aligned = (buf.data_ptr() + 255) // 256 * 256

        def ptr(t):
            return ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _check(self.lib, self.ctx, self.lib.ader_adjoint_lagrangian_step(
            self.ctx, dt, ptr(qs), ptr(xs), ptr(qn), ptr(xn), ptr(qbar), ptr(xbar), ptr(q_next), ptr(x_next),
            ctypes.c_void_p(aligned), n))
        return qbar, xbar, q_next, x_next

    def adjoint_lts(self, n_macro: int, t_end: float, qbar, xbar, keep: int = -1):
        """Gradient through up to n_macro LTS macro steps towards t_end from
        the uploaded state, the schedule held fixed (ader_adjoint_lts): qbar
        (NE, 4) or device [4][NE] and xbar (NV, 2) the adjoints of the final
        averages and positions; keep: macro steps whose cycle states the
        forward keeps (-1: as memory allows; the others are replayed).
        Returns device tensors (qbar0 [4][NE], xbar0 (NV, 2)) and the number
        of macro steps taken; the context ends at the final state."""
        qb = self._dev4(qbar, "qbar")
        xb = self._devxy(xbar, "xbar")
        q0, x0 = self.torch.empty_like(qb), self.torch.empty_like(xb)
        done = ctypes.c_int32()
        _check(self.lib, self.ctx, self.lib.ader_adjoint_lts(
            self.ctx, int(n_macro), int(keep), float(t_end), ctypes.c_void_p(qb.data_ptr()), ctypes.c_void_p(xb.data_ptr()),
            ctypes.c_void_p(q0.data_ptr()), ctypes.c_void_p(x0.data_ptr()), ctypes.byref(done)))
        return q0, x0, done.value

    def probe_contraction(self, F, iters: int, use_mfma: bool):
        """Time `iters` rounds of the predictor's derivative contraction on the
        fields F (device tensor [n][10][6]) on the vector ALUs or the matrix
        cores (ader_probe_contraction); returns (out tensor, milliseconds)."""
        F = F.to(device=self.device, dtype=self.torch.float64).contiguous()
        if F.dim() != 3 or tuple(F.shape[1:]) != (10, 6):
            raise ValueError("F must be [n][10][6]")
        out = self.torch.empty_like(F)
        ms = ctypes.c_float()
        _check(self.lib, self.ctx, self.lib.ader_probe_contraction(
            self.ctx, int(bool(use_mfma)), F.shape[0], iters, ctypes.c_void_p(F.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), ctypes.byref(ms)))
        return out, ms.value

    def set_delta_replay(self, deltas):
        """Macro step m (from the last upload) takes tick length deltas[m]
        (None: the computed ones again)."""
        if deltas is None or len(deltas) == 0:
            _check(self.lib, self.ctx, self.lib.ader_set_delta_replay(self.ctx, None, 0))
            return
        a = np.ascontiguousarray(np.asarray(deltas, np.float64))
        _check(self.lib, self.ctx, self.lib.ader_set_delta_replay(self.ctx, a.ctypes.data_as(ctypes.c_void_p), len(a)))

    def record_schedule(self, steps_per_element: int, macro_steps: int):
        """Record every step each element takes from now on, and each macro
        step's tick length (0: off)."""
        _check(self.lib, self.ctx, self.lib.ader_set_schedule_record(self.ctx, int(steps_per_element),
                                                                     int(macro_steps)))

    def recorded_schedule(self):
        """(step_log, deltas): the steps each element took since recording
        started, and the tick length of every macro step since the upload."""
        ptr = np.zeros(self.NE + 1, np.int32)
        n_steps, n_deltas = ctypes.c_int64(), ctypes.c_int32()
        _check(self.lib, self.ctx, self.lib.ader_get_schedule_record(
            self.ctx, ptr.ctypes.data_as(ctypes.c_void_p), None, 0, None, 0, ctypes.byref(n_steps),
            ctypes.byref(n_deltas)))
        steps = np.zeros(max(n_steps.value, 1), np.int32)
        deltas = np.zeros(max(n_deltas.value, 1), np.float64)
        _check(self.lib, self.ctx, self.lib.ader_get_schedule_record(
            self.ctx, ptr.ctypes.data_as(ctypes.c_void_p), steps.ctypes.data_as(ctypes.c_void_p), len(steps),
            deltas.ctypes.data_as(ctypes.c_void_p), len(deltas), ctypes.byref(n_steps), ctypes.byref(n_deltas)))
        log = [steps[ptr[i]:ptr[i + 1]].tolist() for i in range(self.NE)]
        return log, deltas[:n_deltas.value].tolist()

    def set_schedule_replay(self, step_log):
        """Replay recorded steps: step_log[i] lists the steps (in ticks)
        element i takes, in order (None: the level rule again)."""
        if step_log is None:
            _check(self.lib, self.ctx, self.lib.ader_set_schedule_replay(self.ctx, None, None, 0))
            return
        if len(step_log) != self.NE:
            raise ValueError("one step list per element")
        ptr = np.zeros(self.NE + 1, np.int32)
        ptr[1:] = np.cumsum([len(x) for x in step_log])
        steps = np.ascontiguousarray(np.concatenate([np.asarray(x, np.int64) for x in step_log]).astype(np.int32)) \
            if ptr[-1] else np.zeros(1, np.int32)
        _check(self.lib, self.ctx, self.lib.ader_set_schedule_replay(
            self.ctx, ptr.ctypes.data, steps.ctypes.data, int(ptr[-1])))

    def step_gts(self, t_target, max_steps=0):
        st = _lib.AderStats()
        _check(self.lib, self.ctx, self.lib.ader_step_gts(self.ctx, t_target, max_steps, ctypes.byref(st)))
        return self._stats(st)

    def step_lts(self, t_target, max_macro_steps=0):
        st = _lib.AderStats()
        _check(self.lib, self.ctx, self.lib.ader_step_lts(self.ctx, t_target, max_macro_steps,
                                                          ctypes.byref(st)))
        return self._stats(st)

    def stats(self):
        st = _lib.AderStats()
        _check(self.lib, self.ctx, self.lib.ader_get_stats(self.ctx, ctypes.byref(st)))
        return self._stats(st)

    def download_q(self):
        """The cell averages as a device tensor [4][NE]."""
        Q = self.torch.empty((4, self.NE), dtype=self.torch.float64, device=self.device)
        _check(self.lib, self.ctx, self.lib.ader_download_state(
            self.ctx, ctypes.c_void_p(Q.data_ptr()), None, None))
        return Q

    def download(self):
        """(Q (NE,4), node positions (NV,2), element times (NE,)) as numpy."""
        torch = self.torch
        Q = torch.empty((4, self.NE), dtype=torch.float64, device=self.device)
        X = torch.empty((self.NV, 2), dtype=torch.float64, device=self.device)
        t = torch.empty((self.NE,), dtype=torch.float64, device=self.device)
        _check(self.lib, self.ctx, self.lib.ader_download_state(
            self.ctx, ctypes.c_void_p(Q.data_ptr()), ctypes.c_void_p(X.data_ptr()),
            ctypes.c_void_p(t.data_ptr())))
        return Q.T.cpu().numpy().copy(), X.cpu().numpy(), t.cpu().numpy()

    def inject(self, what, arr):
        dt = np.int32 if what in _lib.INT_ARRAYS else np.float64
        a = np.ascontiguousarray(arr, dt)
        nbytes = self._size(what)
        if a.nbytes != nbytes:
            raise ValueError(f"{what}: {a.nbytes} bytes given, {nbytes} expected")
        _check(self.lib, self.ctx, self.lib.ader_debug_inject(self.ctx, _lib.DBG[what],
                                                              a.ctypes.data, nbytes))

    def autotune(self, trial_macro_steps: int = 2):
        """Time candidate launch settings on the current state (restored afterwards)
        and keep the fastest; returns the choice."""
        t = _lib.AderTune()
        _check(self.lib, self.ctx, self.lib.ader_autotune(self.ctx, trial_macro_steps, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in _lib.AderTune._fields_ if f != "reserved"}

    def set_tune(self, sched_chunk: int = 0, list_wg_per_cu: int = 0, sweep_wg_per_cu: int = 0):
        t = _lib.AderTune(sched_chunk, list_wg_per_cu, 0.0, sweep_wg_per_cu, 0)
        _check(self.lib, self.ctx, self.lib.ader_set_tune(self.ctx, ctypes.byref(t)))

    def instance_times(self):
        """Current time of every instance of a batch."""
        T = np.empty(self.n_instances, np.float64)
        _check(self.lib, self.ctx, self.lib.ader_instance_times(self.ctx, self.n_instances, T.ctypes.data))
        return T

    def set_graphs(self, on: bool):
        """Each macro step as one captured HIP graph (default) or kernel by kernel."""
        _check(self.lib, self.ctx, self.lib.ader_set_graphs(self.ctx, 1 if on else 0))

    def set_profiling(self, on: bool):
        _check(self.lib, self.ctx, self.lib.ader_set_profiling(self.ctx, 1 if on else 0))

    def kernel_times(self):
        """{kernel: (total ms, launches)} since profiling was switched on."""
        n = len(_lib.KERNELS)
        ms = np.zeros(n)
        cnt = np.zeros(n, np.int64)
        _check(self.lib, self.ctx, self.lib.ader_kernel_times(self.ctx, n, ms.ctypes.data, cnt.ctypes.data))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(_lib.KERNELS)}

    def debug_cycles(self, n=1):
        _check(self.lib, self.ctx, self.lib.ader_debug_cycles(self.ctx, n))

    def debug_macro_begin(self, t_end, levels):
        _check(self.lib, self.ctx, self.lib.ader_debug_macro_begin(self.ctx, t_end, levels))
