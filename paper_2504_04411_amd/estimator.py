"""Thin torch-side convenience wrapper over the libhk entry points.

It owns the device buffers (per-set state and the shared workspace, as torch uint8 tensors), uploads
structure-of-arrays inputs and passes raw pointers and the current stream to libhk. Nothing of the
estimator is computed here.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import hk


def _dev(a, device) -> Optional[torch.Tensor]:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)


def _rows(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return [t[i].data_ptr() for i in range(t.shape[0])]


@dataclass
class DevicePhotons:
    """One iteration's light vertices resident on the device, (3, n) float32 tensors."""
    J: int
    pos: torch.Tensor
    flux: torch.Tensor
    nrm: Optional[torch.Tensor] = None
    mis: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    @staticmethod
    def upload(batch, device="cuda") -> "DevicePhotons":
        return DevicePhotons(J=int(batch.J), pos=_dev(batch.pos, device), flux=_dev(batch.flux, device),
                             nrm=_dev(batch.nrm, device), mis=_dev(batch.mis, device))

    def struct(self) -> hk.hk_photons:
        return hk.make_photons(self.J, self.n, _rows(self.pos), _rows(self.flux), _rows(self.nrm), _rows(self.mis))


class Estimator:
    """One libhk context with any number of hit-point sets on one GPU."""

    def __init__(self, r1: float, mode: str = "ppm", device: str = "cuda", stats: str = "luma", **overrides):
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        torch.cuda.set_device(self.device)
        p = hk.hk_default_params(r1)
        p.mode = hk.HK_MODE_VCM if mode == "vcm" else hk.HK_MODE_PPM
        p.stats_channel = hk.HK_STATS_RGB if stats == "rgb" else hk.HK_STATS_LUMA
        self.nch = 3 if stats == "rgb" else 1
        for k, v in overrides.items():
            if v is not None:
                setattr(p, k, v)
        self.params = p
        self.ctx = hk.hk_create(p)
        self.states: Dict[int, torch.Tensor] = {}
        self.n: Dict[int, int] = {}
        self.inputs: Dict[int, list] = {}
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)

    def close(self):
        if self.ctx:
            hk.hk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def _workspace(self, nbytes: int) -> torch.Tensor:
        if self.ws.numel() < nbytes:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.ws

    def set_kernels(self, set_id: int, pos, nrm=None, r_init=None, cam_beta=None, cam_mis=None, r1=None, rmin=None):
        """Uploads a hit-point set; r1 / rmin give the set its own radius scale (default: the context's)."""
        pos_t = _dev(pos, self.device)
        n = int(pos_t.shape[1])
        nrm_t, cb_t, cm_t = _dev(nrm, self.device), _dev(cam_beta, self.device), _dev(cam_mis, self.device)
        r_t = _dev(r_init, self.device)
        st = torch.empty(hk.hk_state_bytes(self.ctx, n), dtype=torch.uint8, device=self.device)
        wsb = hk.hk_workspace_bytes(self.ctx, 0, n)
        ws = self._workspace(wsb)
        hk.hk_set_kernels(self.ctx, set_id, n, -1.0 if r1 is None else r1, -1.0 if rmin is None else rmin,
                          _rows(pos_t), _rows(nrm_t), None if r_t is None else r_t.data_ptr(), _rows(cb_t),
                          _rows(cm_t), st.data_ptr(), ws.data_ptr(), ws.numel(), self.stream)
        self.states[set_id] = st
        self.n[set_id] = n
        self.inputs[set_id] = [pos_t, nrm_t, cb_t, cm_t, r_t]     # kept alive until the stream passes
        return st

    def workspace_for(self, photons: Sequence[DevicePhotons], set_ids: Sequence[int]) -> int:
        return hk.hk_workspace_bytes_batch(self.ctx, [ph.n for ph in photons], [self.n[s] for s in set_ids])

    def iterate(self, set_ids: Sequence[int], photons: Sequence[DevicePhotons]):
        """One iteration of the given sets; their gathers share launches (up to 64 sets each)."""
        wsb = self.workspace_for(photons, set_ids)
        ws = self._workspace(wsb)
        hk.hk_iterate(self.ctx, list(set_ids), [p.struct() for p in photons],
                      [self.states[s].data_ptr() for s in set_ids], ws.data_ptr(), ws.numel(), self.stream)

    def gather_phases(self, set_ids: Sequence[int], photons: Sequence[DevicePhotons]) -> list:
        """Gather phase (0 or 1) of every set within its batch, as an iterate call with these sets
        and light vertices would run them (host-side; nothing is enqueued)."""
        return hk.hk_gather_phases(self.ctx, list(set_ids), [p.struct() for p in photons])

    def capture(self, set_ids: Sequence[int], photons: Sequence[DevicePhotons]) -> "Graph":
        """Captures one iteration of the sets into a graph; refill `photons` in place between launches."""
        wsb = self.workspace_for(photons, set_ids)
        ws = self._workspace(wsb)
        g = hk.hk_graph_create(self.ctx, list(set_ids), [p.struct() for p in photons],
                               [self.states[s].data_ptr() for s in set_ids], ws.data_ptr(), ws.numel())
        return Graph(self, g, ws, list(photons))

    def emit_box(self, set_id: int, scene: hk.hk_box_scene, seed: int, J: int,
                 out: Optional[DevicePhotons] = None) -> DevicePhotons:
        """Generates the set's next batch of J light-vertex slots on the device (hk_emit_box); empty
        slots hold NaN positions. Writes into `out` when given (same J), else into new tensors."""
        vcm = self.params.mode == hk.HK_MODE_VCM
        if out is None:
            mk = lambda: torch.empty((3, J), dtype=torch.float32, device=self.device)  # noqa: E731
            out = DevicePhotons(J=J, pos=mk(), flux=mk(), nrm=mk(), mis=mk() if vcm else None)
        if out.J != J or out.n != J or out.nrm is None or (vcm and out.mis is None):
            raise ValueError("out must hold J slots with normals (and partials for vertex merging)")
        hk.hk_emit_box(self.ctx, set_id, self.states[set_id].data_ptr(), scene, seed, J, _rows(out.pos),
                       _rows(out.nrm), _rows(out.flux), self.stream, mis=_rows(out.mis))
        return out

    def connect_box(self, set_id: int, scene: hk.hk_box_scene, J: int):
        """Adds the vertex-connection term (hk_connect_box) for the iteration about to run."""
        hk.hk_connect_box(self.ctx, set_id, self.states[set_id].data_ptr(), scene, J, self.stream)

    def capture_box(self, set_ids: Sequence[int], scenes, seeds, photons: Sequence[DevicePhotons],
                    connect: bool = False) -> "Graph":
        """Captures generation of every set's batch into `photons` (and, with `connect`, the vertex
        connection) plus one iteration on them: each launch of the graph is one complete iteration."""
        wsb = self.workspace_for(photons, set_ids)
        ws = self._workspace(wsb)
        g = hk.hk_graph_create_box(self.ctx, list(set_ids), list(scenes), list(seeds), [p.struct() for p in photons],
                                   [self.states[s].data_ptr() for s in set_ids], ws.data_ptr(), ws.numel(),
                                   hk.HK_BOX_CONNECT if connect else 0)
        return Graph(self, g, ws, list(photons))

    def autotune(self, set_ids: Sequence[int], photons: Sequence[DevicePhotons]) -> dict:
        """Times the candidate settings on scratch copies of the states and keeps the fastest."""
        wsb = self.workspace_for(photons, set_ids)
        ws = self._workspace(wsb)
        scratch = [torch.empty_like(self.states[s]) for s in set_ids]
        p = hk.hk_autotune(self.ctx, list(set_ids), [ph.struct() for ph in photons],
                           [self.states[s].data_ptr() for s in set_ids], [t.data_ptr() for t in scratch],
                           ws.data_ptr(), ws.numel(), self.stream)
        return dict(cell_scale=p.cell_scale, heavy_cost=p.heavy_cost, lanes_light=p.lanes_light,
                    lanes_heavy=p.lanes_heavy)

    def set_tuning(self, cell_scale=0.0, heavy_cost=0, lanes_light=0, lanes_heavy=0):
        hk.hk_set_tuning(self.ctx, cell_scale, heavy_cost, lanes_light, lanes_heavy)

    def tuning(self) -> dict:
        p = hk.hk_get_params(self.ctx)
        return dict(cell_scale=p.cell_scale, heavy_cost=p.heavy_cost, lanes_light=p.lanes_light,
                    lanes_heavy=p.lanes_heavy)

    # ---- reads (device tensors, original kernel order) -------------------------------------------
    def radiance(self, set_id: int) -> torch.Tensor:
        out = torch.empty((3, self.n[set_id]), dtype=torch.float32, device=self.device)
        hk.hk_read_radiance(self.ctx, set_id, self.states[set_id].data_ptr(), _rows(out), self.stream)
        return out

    def radii(self, set_id: int) -> torch.Tensor:
        out = torch.empty(self.n[set_id], dtype=torch.float32, device=self.device)
        hk.hk_read_radii(self.ctx, set_id, self.states[set_id].data_ptr(), out.data_ptr(), self.stream)
        return out

    def debug(self, set_id: int) -> dict:
        n = self.n[set_id]
        d = dict(count=torch.empty(n, dtype=torch.int32, device=self.device),
                 F=torch.empty(n, dtype=torch.float64, device=self.device),
                 Fc=torch.empty(n, dtype=torch.float64, device=self.device),
                 decision=torch.empty(n, dtype=torch.uint8, device=self.device),
                 t=torch.empty(n, dtype=torch.int32, device=self.device))
        hk.hk_read_debug(self.ctx, set_id, self.states[set_id].data_ptr(), d["count"].data_ptr(), d["F"].data_ptr(),
                         d["Fc"].data_ptr(), d["decision"].data_ptr(), d["t"].data_ptr(), self.stream)
        return d

    def sums(self, set_id: int):
        n = self.n[set_id]
        S = torch.empty((n, 12 * self.nch), dtype=torch.float64, device=self.device)
        Q = torch.empty((n, 12 * self.nch), dtype=torch.float64, device=self.device)
        tau = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        hk.hk_read_sums(self.ctx, set_id, self.states[set_id].data_ptr(), S.data_ptr(), Q.data_ptr(), tau.data_ptr(),
                        self.stream)
        return S, Q, tau

    def stats(self, set_id: int) -> dict:
        out = torch.zeros(4, dtype=torch.int64, device=self.device)
        hk.hk_read_stats(self.ctx, set_id, self.states[set_id].data_ptr(), out.data_ptr(), self.stream)
        v = out.cpu().tolist()
        return dict(iterations=v[0], pairs=v[1], candidates=v[2], cells=v[3])

    def profile(self, on: bool = True):
        hk.hk_profile_enable(self.ctx, on)

    def profile_read(self) -> dict:
        v = hk.hk_profile_read(self.ctx)
        return dict(grid_ms=v[0], fcrit_wait_ms=v[1], list_ms=v[2], gather_ms=v[3], tally_ms=v[4],
                    launches=int(v[5]), gather_ms_phase=[v[6], v[7]], launches_phase=[int(v[8]), int(v[9])])


class Graph:
    """A captured iteration (hk_graph): launch() runs one more iteration of its sets."""

    def __init__(self, est: Estimator, handle: int, ws: torch.Tensor, photons):
        self.est, self.handle, self.ws, self.photons = est, handle, ws, photons

    def launch(self):
        hk.hk_graph_launch(self.handle, self.est.stream)

    def close(self):
        if self.handle:
            hk.hk_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
