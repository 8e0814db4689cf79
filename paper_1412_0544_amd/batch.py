"""Python binding of a batch: many chains advanced by one persistent launch.

Argument marshalling over the C ABI only; the chains are `Chain` objects
whose handles the batch borrows.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .chain import Chain, aligned_empty


class Batch:
    """A persistent-launch batch over `chains` (one model and precision)."""

    def __init__(self, chains: list[Chain], max_steps: int, sites_per_lane: int = 0,
                 kdepth: int = 0, grid_blocks: int = 0, spin_limit: int = 0, flags: int = 0,
                 max_chains: int = 0, max_clusters: int = 0,
                 stream: torch.cuda.Stream | None = None):
        if not chains:
            raise ValueError("a batch needs at least one chain")
        self.chains = list(chains)
        self.device = chains[0].device
        self.desc = L.BatchDesc(int(max_steps), int(max_clusters), int(sites_per_lane), int(kdepth),
                                int(grid_blocks), int(flags), int(spin_limit), int(max_chains))
        n = len(chains)
        self._hs = (L.H * n)(*[c.handle for c in chains])
        lib = L.lib()
        ws = lib.chain_rk4_batch_workspace_bytes(self._hs, n, ctypes.byref(self.desc))
        if ws == 0:
            L.check(L.CHAIN_EINVAL, "chain_rk4_batch_workspace_bytes")
        self._ws, ws_ptr = aligned_empty(ws, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = L.VP()
        L.check(lib.chain_rk4_batch_create(self._hs, n, ctypes.byref(self.desc), ws_ptr, ws,
                                           self.stream.cuda_stream, ctypes.byref(b)),
                "chain_rk4_batch_create")
        self._b = b

    def rebind(self, chains: list[Chain]) -> "Batch":
        """Point the batch at another set of chains within its capacity."""
        n = len(chains)
        hs = (L.H * max(n, 1))(*[c.handle for c in chains])
        L.check(L.lib().chain_rk4_batch_rebind(self._b, hs, n), "chain_rk4_batch_rebind")
        self.chains = list(chains)
        self._hs = hs
        return self

    @staticmethod
    def clusters(n: int, sites_per_lane: int = 0, kdepth: int = 0) -> int:
        """Clusters a chain of n sites takes in a batch of that shape."""
        return int(L.lib().chain_rk4_batch_clusters(int(n), int(sites_per_lane), int(kdepth)))

    def step(self, nsteps) -> "Batch":
        """Advance chain j by nsteps[j] steps (an int applies to every chain)."""
        n = len(self.chains)
        if isinstance(nsteps, int):
            nsteps = [nsteps] * n
        if len(nsteps) != n:
            raise ValueError("one step count per chain")
        arr = (ctypes.c_int64 * n)(*[int(x) for x in nsteps])
        L.check(L.lib().chain_rk4_batch_step(self._b, arr), "chain_rk4_batch_step")
        return self

    def check(self) -> None:
        L.check(L.lib().chain_rk4_batch_check(self._b), "chain_rk4_batch_check")

    def check_status(self) -> int:
        return L.lib().chain_rk4_batch_check(self._b)

    def last_launch(self) -> int:
        """Id of the last launch `step` enqueued (-1 if none)."""
        i = ctypes.c_int64()
        L.check(L.lib().chain_rk4_batch_last_launch(self._b, ctypes.byref(i)),
                "chain_rk4_batch_last_launch")
        return i.value

    def launch_status(self, launch: int) -> int:
        """Wait for one launch (not the ones after it); CHAIN_OK or
        CHAIN_ETIMEOUT (any other status raises)."""
        rc = L.lib().chain_rk4_batch_check_launch(self._b, int(launch))
        if rc not in (L.CHAIN_OK, L.CHAIN_ETIMEOUT):
            L.check(rc, "chain_rk4_batch_check_launch")
        return rc

    @staticmethod
    def plan_for(sites_per_lane: int = 0, kdepth: int = 0, flags: int = 0) -> dict:
        """The shape a batch of these settings uses (no GPU needed)."""
        d = L.BatchDesc(0, 0, int(sites_per_lane), int(kdepth), 0, int(flags), 0, 0)
        P = L.BatchPlan()
        L.check(L.lib().chain_rk4_batch_plan_for(ctypes.byref(d), ctypes.byref(P)),
                "chain_rk4_batch_plan_for")
        return {k: getattr(P, k) for k, _ in L.BatchPlan._fields_}

    @staticmethod
    def layout(n: int, sites_per_lane: int = 0, kdepth: int = 0, flags: int = 0) -> list:
        """How a tiled chain of n sites is cut: (start, keep, wavefronts) per
        cluster (no GPU needed)."""
        d = L.BatchDesc(0, 0, int(sites_per_lane), int(kdepth), 0, int(flags), 0, 0)
        lib = L.lib()
        count = lib.chain_rk4_batch_layout(int(n), ctypes.byref(d), None, None, None, 0)
        if count < 0:
            L.check(L.CHAIN_EINVAL, "chain_rk4_batch_layout")
        start = (ctypes.c_int64 * count)()
        keep = (ctypes.c_int64 * count)()
        waves = (ctypes.c_int32 * count)()
        lib.chain_rk4_batch_layout(int(n), ctypes.byref(d), start, keep, waves, count)
        return [(int(start[i]), int(keep[i]), int(waves[i])) for i in range(count)]

    def energies(self) -> list[float]:
        n = len(self.chains)
        out = (ctypes.c_double * n)()
        L.check(L.lib().chain_rk4_batch_energy(self._b, out), "chain_rk4_batch_energy")
        return list(out)

    def plan(self) -> dict:
        P = L.BatchPlan()
        L.check(L.lib().chain_rk4_batch_get_plan(self._b, ctypes.byref(P)), "chain_rk4_batch_get_plan")
        return {k: getattr(P, k) for k, _ in L.BatchPlan._fields_}

    def close(self) -> None:
        if getattr(self, "_b", None) is not None and self._b.value:
            L.lib().chain_rk4_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
