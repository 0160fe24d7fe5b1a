"""Torch-facing wrapper of the C ABI: device memory and streams from PyTorch,
all computation in the HIP library.

A Solver owns one library context (grid N, batch B, physics) and a cached
workspace tensor.  Fields are float64 CUDA tensors of shape [B, N, N].
"""

import ctypes
from ctypes import byref, c_double, c_int32, c_size_t, c_uint64, c_void_p
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import native as nv

IDENTITY, EXP_ABS, FRACTIONAL, HEAT = 0, 1, 2, 3
VELOCITY, VORTICITY, STREAMFUNCTION = 0, 1, 2


@dataclass(frozen=True)
class KernelSpec:
    """W(|k|): 0 identity, 1 exp(-param|k|), 2 |k|^(-2 param), 3 exp(-param|k|^2)."""
    kind: int = IDENTITY
    param: float = 0.0
    metric: int = VELOCITY

    def c(self):
        return nv.Kernel(self.kind, self.metric, float(self.param))


@dataclass
class Observations:
    """Probe stride, increasing step indices, values [B, n_times, 2, M, M] (device) or None."""
    stride: int
    steps: Sequence[int]
    values: Optional[torch.Tensor] = None

    def c(self):
        arr = (c_int32 * len(self.steps))(*[int(s) for s in self.steps])
        vals = self.values.data_ptr() if self.values is not None else None
        o = nv.Obs(int(self.stride), len(self.steps), ctypes.cast(arr, ctypes.POINTER(c_int32)), vals)
        return o, arr   # keep arr alive while o is used


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, shape, name):
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda):
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _need_bytes(t, nbytes, name):
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.uint8 and t.is_cuda):
        raise TypeError(f"{name} must be a uint8 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < nbytes:
        raise ValueError(f"{name} holds {t.numel()} bytes, needs {nbytes}")


def checkpoint_advances(n_segments, slots):
    """Segment advances of the binomial schedule for n_segments and `slots` snapshot slots (host only)."""
    v = ctypes.c_int64()
    nv.check(nv.load().pa_checkpoint_advances(int(n_segments), int(slots), byref(v)))
    return v.value


def checkpoint_schedule(n_segments, slots):
    """The schedule's actions as (kind, a, b, src, dst) tuples (kind 0 advance, 1 reverse; host only)."""
    lib = nv.load()
    n = ctypes.c_int64()
    nv.check(lib.pa_checkpoint_schedule(int(n_segments), int(slots), None, 0, byref(n)))
    buf = (ctypes.c_int32 * (5 * max(n.value, 1)))()
    nv.check(lib.pa_checkpoint_schedule(int(n_segments), int(slots), buf, n.value, byref(n)))
    return [tuple(buf[5 * i: 5 * i + 5]) for i in range(n.value)]


class Solver:
    def __init__(self, N, B=1, nu=1e-3, dt=5e-3, mu=0.0, forcing_amp=0.0, forcing_k=4,
                 device="cuda", stream: Optional[torch.cuda.Stream] = None):
        self.lib = nv.load()
        self.N, self.B = int(N), int(B)
        self.phys = nv.Physics(float(nu), float(mu), float(dt), float(forcing_amp), int(forcing_k), 0)
        self.device = torch.device(device)
        self.stream = stream
        ctx = c_void_p()
        with torch.cuda.device(self.device):
            nv.check(self.lib.pa_create(byref(self.phys), self.N, self.B, self._stream_handle(), byref(ctx)))
        self.ctx = ctx
        kc = c_int32()
        nv.check(self.lib.pa_get_shape(self.ctx, None, None, byref(kc)))
        self.Kc = kc.value
        self._ws = None
        self._cancel = None

    # ------------------------------------------------------------- plumbing
    def _obs(self, obs: Observations, need_values=False):
        """The C struct of obs (and the step array it points to) after checking that its values,
        which the library reads through a bare pointer, are a contiguous float64 tensor of shape
        [B, n_times, 2, M, M] on the device (M = N / stride)."""
        stride = int(obs.stride)
        if stride < 1 or self.N % stride:
            raise ValueError(f"observation stride {stride} must divide N = {self.N}")
        if obs.values is not None:
            M = self.N // stride
            _need(obs.values, (self.B, len(obs.steps), 2, M, M), "observation values")
        elif need_values:
            raise ValueError("observation values are required")
        return obs.c()

    def _stream_handle(self):
        s = self.stream if self.stream is not None else torch.cuda.current_stream(self.device)
        return c_void_p(s.cuda_stream)

    def _sync_stream(self):
        nv.check(self.lib.pa_set_stream(self.ctx, self._stream_handle()))

    def cancel_flags(self):
        """Host int32 flags [B] bound to this solver (pa_set_cancel_flags), all clear on return:
        setting flags[b] non-zero, from any thread, stops member b of a running assimilate at
        its next iteration boundary with the result of its last completed iteration."""
        if self._cancel is None:
            self._cancel = (c_int32 * self.B)()
            nv.check(self.lib.pa_set_cancel_flags(self.ctx, ctypes.cast(self._cancel, c_void_p)))
        for b in range(self.B):
            self._cancel[b] = 0
        return self._cancel

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, n_steps=0, ckpt_every=1, n_obs=0, lbfgs_m=0):
        b = c_size_t()
        nv.check(self.lib.pa_workspace_bytes(self.ctx, int(n_steps), int(ckpt_every), int(n_obs), int(lbfgs_m),
                                             byref(b)))
        return b.value

    def checkpoint_bytes(self, n_steps, ckpt_every):
        b = c_size_t()
        nv.check(self.lib.pa_checkpoint_bytes(self.ctx, int(n_steps), int(ckpt_every), byref(b)))
        return b.value

    def fit_ckpt_every(self, n_steps, n_obs=0, lbfgs_m=0, budget_bytes=None, reserve=0.1):
        """Largest checkpoint interval K <= n_steps whose workspace fits in budget_bytes.

        The default budget is the device's free memory (plus this solver's
        current workspace, which would be released) less a `reserve` fraction.
        K = n_steps keeps every stage field of the trajectory, so a gradient
        needs no recomputation; smaller K trade recomputation for memory.
        Returns 0 if not even K = 1 fits.
        """
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            held = self._ws.numel() if self._ws is not None else 0
            budget_bytes = int((free + held) * (1.0 - reserve))
        if n_steps <= 1:
            return 1 if self.workspace_bytes(n_steps, 1, n_obs, lbfgs_m) + 256 <= budget_bytes else 0
        for m in range(1, n_steps + 1):
            K = -(-n_steps // m)
            if self.workspace_bytes(n_steps, K, n_obs, lbfgs_m) + 256 <= budget_bytes:
                return K
        return 0

    def set_checkpoint_slots(self, slots):
        """Snapshot budget of the internal checkpoints (pa_set_checkpoint_slots):
        0 keeps one state per segment boundary; 1 <= slots < segments reverses
        the segments with the binomial schedule in that many states."""
        nv.check(self.lib.pa_set_checkpoint_slots(self.ctx, int(slots)))

    def get_checkpoint_slots(self):
        v = ctypes.c_int32()
        nv.check(self.lib.pa_get_checkpoint_slots(self.ctx, byref(v)))
        return v.value

    def fit_checkpointing(self, n_steps, n_obs=0, lbfgs_m=0, budget_bytes=None, reserve=0.1):
        """Segment length K and snapshot budget that fit the workspace in
        budget_bytes with the fewest forward steps.

        Returns (K, slots, forward_steps): slots = 0 when a state per segment
        boundary fits (forward_steps = n_steps + (L - 1) K for L segments),
        else the binomial budget (forward_steps = n_steps + K times the
        schedule's segment advances).  (0, 0, 0) if nothing fits.  The
        default budget is as in fit_ckpt_every.
        """
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            held = self._ws.numel() if self._ws is not None else 0
            budget_bytes = int((free + held) * (1.0 - reserve))
        H = max(int(n_steps), 0)
        if H <= 1:
            K = self.fit_ckpt_every(H, n_obs, lbfgs_m, budget_bytes)
            return (K, 0, H) if K else (0, 0, 0)
        saved = self.get_checkpoint_slots()
        best = None
        try:
            for L in range(1, H + 1):
                K = -(-H // L)
                if L > 1 and -(-H // (L - 1)) == K:
                    continue                    # same K as a smaller L: fewer segments, same store
                L = -(-H // K)
                self.set_checkpoint_slots(0)
                full = self.workspace_bytes(H, K, n_obs, lbfgs_m) + 256
                if full <= budget_bytes:
                    cand = (H + (L - 1) * K, -K, 0)
                else:
                    if L < 2:
                        continue
                    self.set_checkpoint_slots(1)
                    one = self.workspace_bytes(H, K, n_obs, lbfgs_m) + 256
                    if one > budget_bytes:
                        continue
                    self.set_checkpoint_slots(2)
                    per_slot = self.workspace_bytes(H, K, n_obs, lbfgs_m) + 256 - one
                    slots = min(L, 1 + (budget_bytes - one) // max(per_slot, 1))
                    while slots > 1:            # alignment padding: confirm the size
                        self.set_checkpoint_slots(slots)
                        if self.workspace_bytes(H, K, n_obs, lbfgs_m) + 256 <= budget_bytes:
                            break
                        slots -= 1
                    cand = (H + checkpoint_advances(L, slots) * K, -K, slots)
                if best is None or cand < best:
                    best = cand
        finally:
            self.set_checkpoint_slots(saved)
        if best is None:
            return 0, 0, 0
        return -best[1], best[2], best[0]

    def workspace(self, n_steps=0, ckpt_every=1, n_obs=0, lbfgs_m=0):
        need = self.workspace_bytes(n_steps, ckpt_every, n_obs, lbfgs_m)
        if self._ws is None or self._ws.numel() < need + 256:
            self._ws = None
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        return c_void_p(base + off), c_size_t(self._ws.numel() - off)

    def empty(self):
        return torch.empty((self.B, self.N, self.N), dtype=torch.float64, device=self.device)

    def set_tiles(self, **tiles):
        """Tile shapes of the FFT passes (keys of native.TILE_FIELDS; omitted keys keep their value)."""
        unknown = set(tiles) - set(nv.TILE_FIELDS)
        if unknown:
            raise ValueError(f"unknown tile keys {sorted(unknown)}")
        t = nv.Tiles(*[int(tiles.get(k, -1)) for k in nv.TILE_FIELDS])
        nv.check(self.lib.pa_set_tiles(self.ctx, byref(t)))

    def set_sobolev(self, lam):
        """Sobolev regularisation (lambda/2) int |grad u0|^2 of every cost of this solver (pa_set_sobolev)."""
        nv.check(self.lib.pa_set_sobolev(self.ctx, float(lam)))

    def get_tiles(self):
        t = nv.Tiles()
        nv.check(self.lib.pa_get_tiles(self.ctx, byref(t)))
        return {k: getattr(t, k) for k in nv.TILE_FIELDS}

    # ---------------------------------------------------------------- calls
    def init_field(self, seeds, kind=0, k0=4.0, target=0.5, out=None):
        seeds = [int(s) for s in seeds]
        if len(seeds) != self.B:
            raise ValueError("need one seed per member")
        out = self.empty() if out is None else out
        _need(out, (self.B, self.N, self.N), "out")
        arr = (c_uint64 * self.B)(*seeds)
        self._sync_stream()
        ws, wb = self.workspace()
        nv.check(self.lib.pa_init_field(self.ctx, arr, int(kind), float(k0), float(target), _ptr(out), ws, wb))
        return out

    def forward(self, omega0, n_steps, obs: Optional[Observations] = None, want_obs=False, want_J=None,
                ckpt_every=1, ckpt: Optional[torch.Tensor] = None, want_final=True):
        _need(omega0, (self.B, self.N, self.N), "omega0")
        self._sync_stream()
        res = {}
        o_c = None
        keep = None
        if obs is not None:
            o_c, keep = self._obs(obs)
        if ckpt is not None:
            _need_bytes(ckpt, self.checkpoint_bytes(n_steps, ckpt_every), "ckpt")
        if want_J is None:
            want_J = obs is not None and obs.values is not None
        J = torch.empty(self.B, dtype=torch.float64, device=self.device) if want_J else None
        M = self.N // obs.stride if obs is not None else 0
        oo = (torch.empty((self.B, len(obs.steps), 2, M, M), dtype=torch.float64, device=self.device)
              if want_obs else None)
        wT = self.empty() if want_final else None
        ws, wb = self.workspace(0, ckpt_every, len(obs.steps) if obs else 0)
        nv.check(self.lib.pa_forward(self.ctx, _ptr(omega0), int(n_steps), byref(o_c) if o_c else None,
                                     _ptr(J), _ptr(oo), _ptr(wT), int(ckpt_every), _ptr(ckpt), ws, wb))
        del keep
        res["omega_T"] = wT
        res["J"] = J
        res["obs"] = oo
        return res

    def adjoint_gradient(self, omega0, n_steps, obs: Observations, ckpt_every=50):
        _need(omega0, (self.B, self.N, self.N), "omega0")
        self._sync_stream()
        o_c, keep = self._obs(obs, need_values=True)
        J = torch.empty(self.B, dtype=torch.float64, device=self.device)
        g = self.empty()
        ws, wb = self.workspace(n_steps, ckpt_every, len(obs.steps))
        nv.check(self.lib.pa_adjoint_gradient(self.ctx, _ptr(omega0), int(n_steps), byref(o_c), _ptr(J), _ptr(g),
                                              int(ckpt_every), ws, wb))
        del keep
        return J, g

    def adjoint_gradient_noalloc(self, omega0, n_steps, obs: Observations, ckpt_every=50, J=None, grad=None):
        """adjoint_gradient without a workspace (pa_adjoint_gradient_noalloc): the library's own
        per-device scratch holds it, so nothing is allocated when J and grad are given.  Calls
        that overlap on one device race on that scratch."""
        _need(omega0, (self.B, self.N, self.N), "omega0")
        J = torch.empty(self.B, dtype=torch.float64, device=self.device) if J is None else J
        g = self.empty() if grad is None else grad
        _need(J, (self.B,), "J")
        _need(g, (self.B, self.N, self.N), "grad")
        self._sync_stream()
        o_c, keep = self._obs(obs, need_values=True)
        nv.check(self.lib.pa_adjoint_gradient_noalloc(self.ctx, _ptr(omega0), int(n_steps), byref(o_c), _ptr(J),
                                                      _ptr(g), int(ckpt_every)))
        del keep
        return J, g

    def adjoint_from_checkpoints(self, ckpt, n_steps, obs: Observations, ckpt_every, scale=None):
        _need_bytes(ckpt, self.checkpoint_bytes(n_steps, ckpt_every), "ckpt")
        if scale is not None:
            _need(scale, (self.B,), "scale")
        self._sync_stream()
        o_c, keep = self._obs(obs, need_values=True)
        g = self.empty()
        ws, wb = self.workspace(n_steps, ckpt_every, len(obs.steps))
        nv.check(self.lib.pa_adjoint_from_checkpoints(self.ctx, _ptr(ckpt), int(n_steps), byref(o_c), _ptr(scale),
                                                      _ptr(g), int(ckpt_every), ws, wb))
        del keep
        return g

    def precondition(self, x, kernel: KernelSpec, power, out=None):
        _need(x, (self.B, self.N, self.N), "x")
        out = self.empty() if out is None else out
        self._sync_stream()
        k = kernel.c()
        ws, wb = self.workspace()
        nv.check(self.lib.pa_precondition(self.ctx, byref(k), float(power), _ptr(x), _ptr(out), ws, wb))
        return out

    def optimizer_state(self, kernel, method="lbfgs", lbfgs_m=10):
        """A device buffer for the optimiser state of assimilate(..., state_out=...) with this
        kernel argument, method and memory (pa_assimilate_state_bytes); a plain byte image."""
        per_member = not isinstance(kernel, KernelSpec)
        m = int(lbfgs_m) if method == "lbfgs" else 1
        b = c_size_t()
        nv.check(self.lib.pa_assimilate_state_bytes(self.ctx, max(m, 1), int(per_member), byref(b)))
        return torch.empty(b.value, dtype=torch.uint8, device=self.device)

    def assimilate(self, omega_fg, n_steps, obs: Observations, kernel, method="lbfgs",
                   max_iter=10, lbfgs_m=10, ckpt_every=50, state_in=None, state_out=None):
        """4D-Var from the first guess omega_fg [B, N, N].  kernel: one KernelSpec for every
        member, or a sequence of B KernelSpecs (one preconditioner per member: a kernel sweep
        as one batched solve).  Returns (omega0 [B, N, N], J history per member, iterations).
        state_out / state_in (buffers from optimizer_state): write the optimiser state after the
        last iteration / resume from one (omega_fg is then ignored); k iterations written and j
        resumed equal one run of k + j iterations bit for bit (pa_assimilate_ex)."""
        _need(omega_fg, (self.B, self.N, self.N), "omega_fg")
        per_member = not isinstance(kernel, KernelSpec)
        if per_member and len(kernel) != self.B:
            raise ValueError(f"{len(kernel)} kernels for {self.B} members")
        self._sync_stream()
        w = omega_fg.clone()
        o_c, keep = self._obs(obs, need_values=True)
        hist = (c_double * (self.B * (max_iter + 1)))()
        iters = (c_int32 * self.B)()
        m = int(lbfgs_m) if method == "lbfgs" else 1
        ws, wb = self.workspace(n_steps, ckpt_every, len(obs.steps), max(m, 1))
        meth = 0 if method == "lbfgs" else 1
        if state_in is not None or state_out is not None:
            states = [t for t in (state_in, state_out) if t is not None]
            idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
            for t in states:
                if t.dtype != torch.uint8 or t.device != torch.device("cuda", idx) or not t.is_contiguous():
                    raise ValueError("optimiser states are contiguous uint8 tensors on the solver's device")
            sb = min(t.numel() for t in states)
            ks = (nv.Kernel * self.B)(*[k.c() for k in kernel]) if per_member else (nv.Kernel * 1)(kernel.c())
            nv.check(self.lib.pa_assimilate_ex(self.ctx, _ptr(w), int(n_steps), byref(o_c), ks, int(per_member),
                                               meth, int(max_iter), m, int(ckpt_every), hist, iters,
                                               _ptr(state_in) if state_in is not None else None,
                                               _ptr(state_out) if state_out is not None else None, sb, ws, wb))
        elif per_member:
            ks = (nv.Kernel * self.B)(*[k.c() for k in kernel])
            nv.check(self.lib.pa_assimilate_kernels(self.ctx, _ptr(w), int(n_steps), byref(o_c), ks, meth,
                                                    int(max_iter), m, int(ckpt_every), hist, iters, ws, wb))
        else:
            k = kernel.c()
            nv.check(self.lib.pa_assimilate(self.ctx, _ptr(w), int(n_steps), byref(o_c), byref(k), meth,
                                            int(max_iter), m, int(ckpt_every), hist, iters, ws, wb))
        del keep
        H = [[hist[b * (max_iter + 1) + i] for i in range(max_iter + 1)] for b in range(self.B)]
        return w, H, [iters[b] for b in range(self.B)]

    def assimilate_members(self, omega_fg, obs, kernels, method="lbfgs", max_iter=10, lbfgs_m=10, ckpt_every=50):
        """4D-Var of B independent problems that share the grid and physics but not their
        observations (pa_assimilate_members): obs is a list of B Observations, each with its own
        stride, steps and values [1, n_times, 2, M, M]; kernels a list of B KernelSpecs.  A
        member's horizon is its last observation step; each member's result is that of a solve
        of it alone over its own horizon.  Returns (omega0 [B, N, N], J histories, iterations)."""
        _need(omega_fg, (self.B, self.N, self.N), "omega_fg")
        if len(obs) != self.B or len(kernels) != self.B:
            raise ValueError(f"need {self.B} observation sets and kernels")
        keep, sets = [], []
        for o in obs:
            stride = int(o.stride)
            if stride < 1 or self.N % stride:
                raise ValueError(f"observation stride {stride} must divide N = {self.N}")
            M = self.N // stride
            _need(o.values, (1, len(o.steps), 2, M, M), "observation values")
            c_o, arr = o.c()
            keep.append(arr)
            sets.append(c_o)
        n_steps = max(int(o.steps[-1]) for o in obs)
        self._sync_stream()
        w = omega_fg.clone()
        obs_arr = (nv.Obs * self.B)(*sets)
        ks = (nv.Kernel * self.B)(*[k.c() for k in kernels])
        hist = (c_double * (self.B * (max_iter + 1)))()
        iters = (c_int32 * self.B)()
        m = int(lbfgs_m) if method == "lbfgs" else 1
        ws, wb = self.workspace(n_steps, ckpt_every, max(len(o.steps) for o in obs), max(m, 1))
        nv.check(self.lib.pa_assimilate_members(self.ctx, _ptr(w), int(n_steps), obs_arr, ks,
                                                0 if method == "lbfgs" else 1, int(max_iter), m, int(ckpt_every),
                                                hist, iters, ws, wb))
        del keep
        H = [[hist[b * (max_iter + 1) + i] for i in range(max_iter + 1)] for b in range(self.B)]
        return w, H, [iters[b] for b in range(self.B)]

    def adjoint_impulse(self, omega0, n_steps, ix, iy, n_shells, ckpt_every=50, want_field=False, acc=None):
        """Impulse response shells [B][n_steps + 1][n_shells] (and P lambda_0 if want_field);
        with acc (an EnsembleAccumulator), the batch is added to its ensemble sums."""
        _need(omega0, (self.B, self.N, self.N), "omega0")
        self._sync_stream()
        sh = torch.empty((self.B, n_steps + 1, n_shells), dtype=torch.float64, device=self.device)
        f = self.empty() if want_field else None
        ws, wb = self.workspace(n_steps, ckpt_every, 0)
        if acc is not None:
            acc.check(self, n_steps, n_shells)
        nv.check(self.lib.pa_adjoint_impulse(self.ctx, _ptr(omega0), int(n_steps), int(ix), int(iy), int(n_shells),
                                             _ptr(sh), _ptr(f), byref(acc.c) if acc is not None else None,
                                             int(ckpt_every), ws, wb))
        return sh, f

    def ensemble_accumulator(self, n_steps, n_shells):
        return EnsembleAccumulator(self, n_steps, n_shells)

    def ensemble_stats(self, acc, rows=None):
        """Ensemble statistics (pa_ensemble_stats) of the members accumulated in acc, per backward step."""
        rows = acc.rows if rows is None else int(rows)
        z = lambda *shape: torch.empty(shape, dtype=torch.float64, device=self.device)
        out = {"mean_energy": z(rows, acc.n_shells), "energy_of_mean": z(rows, acc.n_shells),
               "total_mean": z(rows), "total_of_mean": z(rows), "snr": z(rows)}
        self._sync_stream()
        nv.check(self.lib.pa_ensemble_stats(self.ctx, byref(acc.c), rows, acc.n_shells, _ptr(out["mean_energy"]),
                                            _ptr(out["energy_of_mean"]), _ptr(out["total_mean"]),
                                            _ptr(out["total_of_mean"]), _ptr(out["snr"])))
        out["members"] = acc.count
        return out

    # ----------------------------------------------------------- measurement
    def profile_start(self, kernel_class, sample_every=1):
        """Time every sample_every-th launch of a kernel class with HIP events
        on this solver's stream (0 row rhs, 1 column forward, 2 row adjoint,
        3 column adjoint)."""
        self._sync_stream()
        nv.check(self.lib.pa_profile_start(self.ctx, int(kernel_class), int(sample_every)))

    def profile_stop(self):
        t = ctypes.c_int64()
        seen = ctypes.c_int64()
        ms = c_double()
        nv.check(self.lib.pa_profile_stop(self.ctx, byref(t), byref(seen), byref(ms)))
        return {"timed_launches": t.value, "launches": seen.value, "total_ms": ms.value}

    # ---------------------------------------------------------- extra calls
    def first_guess(self, stride, probes, out=None):
        """Interpolated vorticity from probe velocities probes [B, 2, M, M] at t = 0."""
        M = self.N // int(stride)
        _need(probes, (self.B, 2, M, M), "probes")
        out = self.empty() if out is None else out
        self._sync_stream()
        ws, wb = self.workspace()
        nv.check(self.lib.pa_first_guess(self.ctx, int(stride), _ptr(probes), _ptr(out), ws, wb))
        return out

    def shell_growth(self, shells, tau_min=0.3, tau_max=1.0):
        """Member mean of shells [B, rows, n] and per-shell growth rate of ln(mean) vs tau."""
        B, rows, n = shells.shape
        if B != self.B or shells.dtype != torch.float64 or not shells.is_cuda or not shells.is_contiguous():
            raise ValueError("shells must be a contiguous float64 CUDA tensor [B, rows, n_shells]")
        mean = torch.empty((rows, n), dtype=torch.float64, device=self.device)
        rate = torch.empty(n, dtype=torch.float64, device=self.device)
        self._sync_stream()
        nv.check(self.lib.pa_shell_growth(self.ctx, _ptr(shells), int(rows), int(n), float(tau_min), float(tau_max),
                                          _ptr(mean), _ptr(rate)))
        return mean, rate


class EnsembleAccumulator:
    """Device running sums of an ensemble of impulse responses (pa_ensemble_acc):
    member sum of the adjoint state per backward step, of the total adjoint energy
    and of the shell energies.  Add batches with Solver.adjoint_impulse(..., acc=...)
    (any solver of the same grid size), read statistics with Solver.ensemble_stats."""

    def __init__(self, solver, n_steps, n_shells):
        lb, eb, sb = c_size_t(), c_size_t(), c_size_t()
        nv.check(solver.lib.pa_ensemble_acc_bytes(solver.ctx, int(n_steps), int(n_shells), byref(lb), byref(eb),
                                                  byref(sb)))
        dev = solver.device
        self.N, self.n_steps, self.n_shells, self.rows = solver.N, int(n_steps), int(n_shells), int(n_steps) + 1
        self.lambda_sum = torch.zeros(lb.value, dtype=torch.uint8, device=dev)
        self.energy_sum = torch.zeros(eb.value // 8, dtype=torch.float64, device=dev)
        self.shell_sum = torch.zeros(sb.value // 8, dtype=torch.float64, device=dev)
        self.c = nv.EnsembleAcc(self.lambda_sum.data_ptr(), self.energy_sum.data_ptr(), self.shell_sum.data_ptr(), 0)

    @property
    def count(self):
        return self.c.count

    def check(self, solver, n_steps, n_shells):
        if solver.N != self.N or int(n_steps) != self.n_steps or int(n_shells) != self.n_shells:
            raise ValueError("accumulator made for another grid size, horizon or shell count")

