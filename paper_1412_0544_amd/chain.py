"""Python binding of one chain: argument marshalling over the C ABI only.

Torch supplies the device memory (state and workspace) and the stream; every
step of the integration runs in the HIP library.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

MODELS = {"quartic": L.CHAIN_QUARTIC, "harmonic": L.CHAIN_HARMONIC,
          "quartic_nnn": L.CHAIN_QUARTIC_NNN, "harmonic_nnn": L.CHAIN_HARMONIC_NNN}
PRECS = {"fp64": L.CHAIN_FP64, "fp32_kahan": L.CHAIN_FP32_KAHAN,
         "fp32_kahan64": L.CHAIN_FP32_KAHAN64, "fp32": L.CHAIN_FP32}
METHODS = {"fused": L.CHAIN_FUSED, "naive": L.CHAIN_NAIVE}


def _code(table, v):
    if isinstance(v, str):
        return table[v]
    return int(v)


def state_dtype(prec) -> torch.dtype:
    return torch.float64 if _code(PRECS, prec) == L.CHAIN_FP64 else torch.float32


def aligned_empty(nbytes: int, device, align: int = 256) -> tuple[torch.Tensor, int]:
    """A byte tensor holding at least nbytes at an `align`-aligned address."""
    buf = torch.empty(max(1, nbytes + align), dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % align
    return buf, buf.data_ptr() + off


def make_tableau(a, b) -> L.Tableau:
    """The C struct of a Butcher tableau from nested sequences."""
    s = len(b)
    if s < 1 or s > L.CHAIN_MAX_STAGES or len(a) != s or any(len(r) != s for r in a):
        raise ValueError(f"a must be s x s and b of length s, 1 <= s <= {L.CHAIN_MAX_STAGES}")
    t = L.Tableau()
    t.stages = s
    for j in range(s):
        t.b[j] = float(b[j])
        for m in range(j):
            t.a[j][m] = float(a[j][m])
    return t


def tableau_reach(model, a, b) -> int:
    """Sites per side one step of the method reaches for the model."""
    r = L.lib().chain_rk4_tableau_reach(_code(MODELS, model), ctypes.byref(make_tableau(a, b)))
    if r < 0:
        L.check(L.CHAIN_EINVAL, "chain_rk4_tableau_reach")
    return int(r)


def plan_for(n: int, dt: float = 0.01, model="quartic", prec="fp64", method="fused",
             sites_per_lane: int = 0, kdepth: int = 0, waves_per_cluster: int = 0,
             flags: int = 0, tableau=None) -> dict:
    """The plan the library gives a chain of these settings (no GPU needed);
    ``tableau`` is (a, b) of an explicit method, as for ``Chain``."""
    scheme = L.CHAIN_SCHEME_RK4 if tableau is None else L.CHAIN_SCHEME_TABLEAU
    d = L.Desc(int(n), _code(MODELS, model), _code(PRECS, prec), float(dt), _code(METHODS, method),
               int(sites_per_lane), int(kdepth), int(waves_per_cluster), int(flags), scheme)
    t = None if tableau is None else ctypes.byref(make_tableau(*tableau))
    P = L.Plan()
    L.check(L.lib().chain_rk4_plan_for(ctypes.byref(d), t, ctypes.byref(P)), "chain_rk4_plan_for")
    return {k: getattr(P, k) for k, _ in L.Plan._fields_}


class Chain:
    """One periodic chain advanced by the HIP library.

    ``q0`` and ``p0`` (numpy arrays or tensors) are copied into device tensors
    of the precision's dtype; ``state()`` returns those tensors.

    model: "quartic", "harmonic", "quartic_nnn" or "harmonic_nnn";
    prec: "fp64", "fp32_kahan", "fp32_kahan64" (FP32 state, FP64 carries) or
    "fp32" (no compensation, a control); the last two run classical RK4 on
    a single tiled chain only. method: "fused" or "naive" (one kernel per
    stage). sites_per_lane, waves_per_cluster and kdepth fix the cluster
    shape (0 = the library's plan for this length). graph: replay each
    distinct step count from a captured graph (saves launch time on short
    chains). resident: True keeps a ring of at most 4096 sites in one
    workgroup for all steps of a call. tableau: (a, b) of any explicit
    Runge-Kutta method instead of classical RK4 (see ``tableaus``).
    """

    def __init__(self, q0, p0, dt: float, model="quartic", prec="fp64", method="fused",
                 sites_per_lane: int = 0, kdepth: int = 0, waves_per_cluster: int = 0,
                 graph: bool = False,
                 resident: bool | None = None, device="cuda",
                 stream: torch.cuda.Stream | None = None,
                 tableau=None):
        self.device = torch.device(device)
        dtype = state_dtype(prec)
        self.q = torch.as_tensor(q0).to(device=self.device, dtype=dtype).contiguous().clone()
        self.p = torch.as_tensor(p0).to(device=self.device, dtype=dtype).contiguous().clone()
        if self.q.ndim != 1 or self.q.shape != self.p.shape:
            raise ValueError("q0 and p0 must be 1-D of one length")
        # resident: None = the library plan (tiled), True = the ring stays in
        # one workgroup for all steps of a call, False = tiled
        flags = ((L.CHAIN_FLAG_GRAPH if graph else 0) |
                 {None: 0, True: L.CHAIN_FLAG_RESIDENT, False: L.CHAIN_FLAG_NO_RESIDENT}[resident])
        scheme = L.CHAIN_SCHEME_RK4 if tableau is None else L.CHAIN_SCHEME_TABLEAU
        self.prec = _code(PRECS, prec)
        self.desc = L.Desc(self.q.numel(), _code(MODELS, model), self.prec, float(dt),
                           _code(METHODS, method), int(sites_per_lane), int(kdepth),
                           int(waves_per_cluster), flags, scheme)
        lib = L.lib()
        ws = lib.chain_rk4_workspace_bytes(ctypes.byref(self.desc))
        if ws == 0:
            L.check(L.CHAIN_EINVAL, "chain_rk4_workspace_bytes")
        self._ws, ws_ptr = aligned_empty(ws, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = L.H()
        L.check(lib.chain_rk4_create(ctypes.byref(self.desc), self.q.data_ptr(), self.p.data_ptr(),
                                     ws_ptr, ws, self.stream.cuda_stream, ctypes.byref(h)),
                "chain_rk4_create")
        self._h = h
        if tableau is not None:
            self.set_tableau(*tableau)

    @property
    def handle(self):
        return self._h

    def set_tableau(self, a, b) -> None:
        """Give the chain an explicit Runge-Kutta method: coefficients ``a``
        (s x s, strictly lower triangle used) and weights ``b`` (s)."""
        L.check(L.lib().chain_rk4_set_tableau(self._h, ctypes.byref(make_tableau(a, b))),
                "chain_rk4_set_tableau")

    def step(self, nsteps: int) -> "Chain":
        L.check(L.lib().chain_rk4_step(self._h, int(nsteps)), "chain_rk4_step")
        return self

    def check(self) -> None:
        """Synchronise the chain's stream (``chain_rk4_check``)."""
        L.check(L.lib().chain_rk4_check(self._h), "chain_rk4_check")

    def energy(self) -> float:
        e = ctypes.c_double()
        L.check(L.lib().chain_rk4_energy(self._h, ctypes.byref(e)), "chain_rk4_energy")
        return e.value

    def set_stream(self, stream: torch.cuda.Stream) -> None:
        L.check(L.lib().chain_rk4_set_stream(self._h, stream.cuda_stream), "chain_rk4_set_stream")
        self.stream = stream

    def plan(self) -> dict:
        P = L.Plan()
        L.check(L.lib().chain_rk4_get_plan(self._h, ctypes.byref(P)), "chain_rk4_get_plan")
        return {k: getattr(P, k) for k, _ in L.Plan._fields_}

    def carries(self):
        """Device pointers (ints) of the carries, or (None, None) for FP64."""
        cq, cp = L.VP(), L.VP()
        L.check(L.lib().chain_rk4_get_carries(self._h, ctypes.byref(cq), ctypes.byref(cp)),
                "chain_rk4_get_carries")
        return cq.value, cp.value

    def carry_tensors(self):
        """Views of the carries as tensors (float32, or float64 for
        "fp32_kahan64"); (None, None) for FP64."""
        cq, cp = self.carries()
        if cq is None:
            return None, None
        base = self._ws.data_ptr()
        n = self.q.numel()
        dt = torch.float64 if self.prec == L.CHAIN_FP32_KAHAN64 else torch.float32
        w = 8 if dt == torch.float64 else 4
        flat = self._ws.view(torch.uint8)
        tq = flat[cq - base: cq - base + w * n].view(dt)
        tp = flat[cp - base: cp - base + w * n].view(dt)
        return tq, tp

    def state(self):
        return self.q, self.p

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            L.lib().chain_rk4_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RoesslerChain:
    """The Roessler chain (three FP64 coordinates per site) advanced by the
    HIP library; ``x``, ``y``, ``z`` are the device state tensors. There is no
    energy (the system is dissipative) and no batching."""

    def __init__(self, x0, y0, z0, dt: float, method="fused", sites_per_lane: int = 0,
                 kdepth: int = 0, waves_per_cluster: int = 0, graph: bool = False,
                 device="cuda", stream: torch.cuda.Stream | None = None,
                 exchange: bool = False):
        self.device = torch.device(device)
        as_dev = lambda a: torch.as_tensor(a).to(device=self.device,  # noqa: E731
                                                 dtype=torch.float64).contiguous().clone()
        self.x, self.y, self.z = as_dev(x0), as_dev(y0), as_dev(z0)
        if self.x.ndim != 1 or self.x.shape != self.y.shape or self.x.shape != self.z.shape:
            raise ValueError("x0, y0 and z0 must be 1-D of one length")
        # exchange: every cluster stays in registers for a whole step call,
        # swapping only edge sites between passes (the whole chain must fit)
        flags = (L.CHAIN_FLAG_GRAPH if graph else 0) | (L.CHAIN_FLAG_EXCHANGE if exchange else 0)
        self.desc = L.Desc(self.x.numel(), L.CHAIN_ROESSLER, L.CHAIN_FP64, float(dt),
                           _code(METHODS, method), int(sites_per_lane), int(kdepth),
                           int(waves_per_cluster), flags, 0)
        lib = L.lib()
        ws = lib.chain_rk4_workspace_bytes(ctypes.byref(self.desc))
        if ws == 0:
            L.check(L.CHAIN_EINVAL, "chain_rk4_workspace_bytes")
        self._ws, ws_ptr = aligned_empty(ws, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = L.H()
        L.check(lib.chain_rk4_create3(ctypes.byref(self.desc), self.x.data_ptr(),
                                      self.y.data_ptr(), self.z.data_ptr(), ws_ptr, ws,
                                      self.stream.cuda_stream, ctypes.byref(h)),
                "chain_rk4_create3")
        self._h = h

    @property
    def handle(self):
        return self._h

    def step(self, nsteps: int) -> "RoesslerChain":
        L.check(L.lib().chain_rk4_step(self._h, int(nsteps)), "chain_rk4_step")
        return self

    def check(self) -> None:
        """Synchronise; raise if a step call's wait for neighbours timed out."""
        L.check(L.lib().chain_rk4_check(self._h), "chain_rk4_check")

    def plan(self) -> dict:
        P = L.Plan()
        L.check(L.lib().chain_rk4_get_plan(self._h, ctypes.byref(P)), "chain_rk4_get_plan")
        return {k: getattr(P, k) for k, _ in L.Plan._fields_}

    def state(self):
        return self.x, self.y, self.z

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            L.lib().chain_rk4_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def energy_noalloc(q: torch.Tensor, p: torch.Tensor, model="quartic", prec="fp64", cq=None,
                   cp=None, stream: torch.cuda.Stream | None = None) -> float:
    """Energy of a state in device tensors without a handle or workspace
    (``chain_rk4_energy_noalloc``: the library allocates nothing); the same
    bits as ``Chain.energy`` over the same state."""
    stream = stream if stream is not None else torch.cuda.current_stream(q.device)
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    e = ctypes.c_double()
    L.check(L.lib().chain_rk4_energy_noalloc(_code(MODELS, model), _code(PRECS, prec), q.numel(),
                                             ptr(q), ptr(p), ptr(cq), ptr(cp), stream.cuda_stream,
                                             ctypes.byref(e)),
            "chain_rk4_energy_noalloc")
    return e.value
