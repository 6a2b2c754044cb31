"""Batched ensembles: many simulations of any size and precision advanced
together through the library's batch API (one launch per kernel group per
step over all members' tiles, runs of steps captured in a HIP graph).
Large members without a sweep window are stepped by their own launches
instead (see ``Ensemble``)."""
from __future__ import annotations

import ctypes

from . import _ffi
from .sim import Sim, _torch


def tiles(cfg: dict) -> int:
    """Thread blocks per step of a simulation with this workload dict."""
    p = _ffi.make_params(cfg)
    return int(_ffi.lib().lbm_tiles(ctypes.byref(p)))


class Ensemble:
    """A set of ``Sim`` members stepped together on one stream.

    Members are created on the ensemble's own stream (a fresh, default-
    priority torch stream unless one is given), which the graph capture needs.

    Members of at least ``solo_min_sites`` sites without a sweep window are
    stepped by their own kernel launches, one after another on the same
    stream, and the rest through the batch: a step of such a member keeps the
    GPU busy long enough (over 40 us) for its launch to cost nothing, and the
    solo kernels run them faster (on MI355X 73-78% of the HBM peak against
    67-68% in the batch for 1024 x 4096 and 2048 x 8192 members).  Results
    are the same bit for bit either way.  None batches every member.
    """

    def __init__(self, cfgs=(), device: str = "cuda:0", stream=None, max_members: int = 1024,
                 max_tiles: int | None = None, solo_min_sites: int | None = 1 << 22):
        torch = _torch()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._lib = _ffi.lib()
        cfgs = list(cfgs)
        self.max_members = max(int(max_members), len(cfgs))
        if max_tiles is None:
            max_tiles = max(1 << 20, sum(tiles(c) for c in cfgs))
        self.max_tiles = int(max_tiles)
        nbytes = int(self._lib.lbm_batch_workspace_bytes(self.max_members, self.max_tiles))
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        b = ctypes.c_void_p()
        rc = self._lib.lbm_batch_create(ctypes.c_void_p(self._ws.data_ptr()), nbytes,
                                        self.max_members, self.max_tiles,
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b))
        if rc != 0:
            raise _ffi.LbmError(rc, "lbm_batch_create")
        self._b = b
        self.solo_min_sites = solo_min_sites
        self.members: list[Sim] = []
        self._solo: list[Sim] = []      # members stepped by their own launches
        for c in cfgs:
            self.add(c)

    @property
    def stepped_alone(self) -> list[Sim]:
        """The members stepped by their own launches."""
        return list(self._solo)

    def _steps_alone(self, sim: Sim) -> bool:
        c = sim.cfg
        return (self.solo_min_sites is not None and not c.get("window", False)
                and int(c["L"]) * int(c["H"]) >= self.solo_min_sites)

    def new_member(self, cfg: dict) -> Sim:
        """Create a Sim on the ensemble's stream (not yet a member)."""
        return Sim(cfg, device=str(self.device), stream=self.stream)

    def add(self, cfg_or_sim) -> Sim:
        sim = cfg_or_sim if isinstance(cfg_or_sim, Sim) else self.new_member(cfg_or_sim)
        if self._steps_alone(sim):
            self._solo.append(sim)
        else:
            rc = self._lib.lbm_batch_add(self._b, sim.handle)
            if rc != 0:
                raise _ffi.LbmError(rc, "lbm_batch_add")
        self.members.append(sim)
        return sim

    def remove(self, sim: Sim) -> None:
        if sim in self._solo:
            self._solo.remove(sim)
        else:
            rc = self._lib.lbm_batch_remove(self._b, sim.handle)
            if rc != 0:
                raise _ffi.LbmError(rc, "lbm_batch_remove")
        self.members.remove(sim)

    def step(self, n: int = 1) -> None:
        rc = self._lib.lbm_batch_step(self._b, int(n))
        if rc != 0:
            raise _ffi.LbmError(rc, "lbm_batch_step")
        for sim in self._solo:
            try:
                sim.step(n)
            except _ffi.LbmError as e:
                # a member whose fault has been reported keeps it to itself,
                # as a batch member does
                if e.code != _ffi.E_STATE:
                    raise

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if getattr(self, "_b", None):
            self._lib.lbm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
