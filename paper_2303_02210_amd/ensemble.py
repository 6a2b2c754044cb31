"""Batched ensembles: many simulations of any size and precision advanced
together through the library's batch API (one launch per kernel group per
step over all members' tiles, large members by their own launches, runs of
steps captured in one HIP graph)."""
from __future__ import annotations

import ctypes

from . import _ffi
from .sim import Sim, _torch


def tiles(cfg: dict) -> int:
    """Thread blocks per step of a simulation with this workload dict."""
    p = _ffi.make_params(cfg)
    return int(_ffi.lib().lbm_tiles(ctypes.byref(p)))


class Ensemble:
    """A set of ``Sim`` members stepped together on one stream, all through
    one batch (one graph launch per run of steps).

    Members are created on the ensemble's own stream (a fresh, default-
    priority torch stream unless one is given), which the graph capture needs.

    Members of at least ``solo_min_sites`` sites that do not move their wall
    or window and do not grow by a division law are stepped inside the batch's
    graph by their own launches of the solo kernels (LBM_FLAG_BATCH_OWN), the
    rest through the shared tile table: a step of such a member keeps the GPU
    busy long enough for its launch to cost nothing, and the solo kernels run
    them faster than the table (on MI355X 73-78% of the HBM peak against
    67-68% for 1024 x 4096 and 2048 x 8192 members).  Results are the same bit
    for bit either way.  None steps every member through the table.

    ``persistent``: each table group whose members neither move their wall or
    window nor grow by a division law runs a whole ``step(n)`` in one
    cooperative launch with a grid-wide barrier between steps, instead of
    one launch per step replayed from a graph (lbm_batch_persistent).
    """

    def __init__(self, cfgs=(), device: str = "cuda:0", stream=None, max_members: int = 1024,
                 max_tiles: int | None = None, solo_min_sites: int | None = 1 << 22,
                 persistent: bool = False):
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
        if persistent:
            rc = self._lib.lbm_batch_persistent(self._b, 1)
            if rc != 0:
                raise _ffi.LbmError(rc, "lbm_batch_persistent")
        self.persistent = bool(persistent)
        self.solo_min_sites = solo_min_sites
        self.members: list[Sim] = []
        for c in cfgs:
            self.add(c)

    @staticmethod
    def _can_step_alone(cfg: dict) -> bool:
        return (not cfg.get("window", False) and cfg.get("ybc", "fixed") != "follow"
                and not str(cfg.get("growth", "bulk")).startswith("division"))

    def _placed(self, cfg: dict) -> dict:
        """cfg with the batch placement flag the ensemble's threshold asks for."""
        if "batch_own" in cfg or "batch_table" in cfg:
            return cfg
        big = (self.solo_min_sites is not None and self._can_step_alone(cfg)
               and int(cfg["L"]) * int(cfg["H"]) >= self.solo_min_sites)
        return dict(cfg, batch_own=True) if big else dict(cfg, batch_table=True)

    @property
    def stepped_alone(self) -> list[Sim]:
        """The members stepped by their own launches inside the batch's graph."""
        out = []
        for m in self.members:
            c = m.cfg
            if c.get("batch_table", False) or not self._can_step_alone(c):
                continue
            if c.get("batch_own", False) or int(c["L"]) * int(c["H"]) >= (1 << 22):
                out.append(m)
        return out

    def new_member(self, cfg: dict) -> Sim:
        """Create a Sim on the ensemble's stream (not yet a member)."""
        return Sim(self._placed(cfg), device=str(self.device), stream=self.stream)

    def add(self, cfg_or_sim) -> Sim:
        sim = cfg_or_sim if isinstance(cfg_or_sim, Sim) else self.new_member(cfg_or_sim)
        rc = self._lib.lbm_batch_add(self._b, sim.handle)
        if rc != 0:
            raise _ffi.LbmError(rc, "lbm_batch_add (a member must use the ensemble's stream)")
        self.members.append(sim)
        return sim

    def remove(self, sim: Sim) -> None:
        rc = self._lib.lbm_batch_remove(self._b, sim.handle)
        if rc != 0:
            raise _ffi.LbmError(rc, "lbm_batch_remove")
        self.members.remove(sim)

    def step(self, n: int = 1) -> None:
        """n steps of every member (LBM_E_STATE if a member has latched a
        fault: remove it and step again)."""
        rc = self._lib.lbm_batch_step(self._b, int(n))
        if rc != 0:
            raise _ffi.LbmError(rc, "lbm_batch_step")

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
