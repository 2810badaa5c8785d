"""Helpers for the GPU parity tests: run HIP stages through the C ABI on seeded
workloads and bring slot-ordered results back in particle-id order."""
import numpy as np
import torch

import oracle
from paper_2005_02656_amd import sph


def configs(w, **kw):
    """(GPU config, oracle config) for a workload, sharing its parameters."""
    g = sph.Config.from_params(w.n, w.params, **kw)
    keys = set(oracle.Config.__dataclass_fields__)
    o = oracle.Config(**{k: v for k, v in g.__dict__.items() if k in keys})
    return g, o


class Run:
    """One workload on the GPU: particles, workspace, globals."""

    def __init__(self, w, cfg, arrays=None):
        self.w = w
        self.cfg = cfg
        self.parts = sph.Particles.from_arrays(arrays if arrays is not None else w.arrays, cfg)
        self.ws = sph.Workspace(cfg)
        self.g = sph.Globals()
        sph.workspace_init(cfg, self.ws)

    def ids(self):
        return self.parts["id"].cpu().numpy()

    def by_id(self, field):
        v = self.parts[field].cpu().numpy()
        out = np.empty_like(v)
        out[self.ids()] = v
        return out

    def put_by_id(self, field, values):
        """Upload an id-ordered array into the slot order of the device arrays."""
        v = np.asarray(values, dtype=np.float64)[self.ids()]
        self.parts[field] = torch.from_numpy(v).to(self.parts[field].device)

    def status(self):
        return sph.status_sync(self.ws)

    def neighbor_pairs(self):
        """Sorted (id_a, id_b, in_gather) triples of every list entry."""
        nc, ns, lst = sph.neighbors_view(self.cfg, self.ws)
        nc = nc.cpu().numpy().astype(np.int64)
        ns = ns.cpu().numpy().astype(np.int64)
        lst = lst.cpu().numpy()                     # (tiles, ng_max, 64)
        ids = self.ids()
        ng = self.cfg.ng_max
        n = ids.size
        rows = []
        for j in range(ng):
            col = lst[:, j, :].reshape(-1)[:n]      # entry j of every slot
            a_g = np.nonzero(j < nc)[0]
            rows.append(np.stack([ids[a_g], ids[col[a_g]], np.ones_like(a_g)], 1))
            a_s = np.nonzero(j >= ng - (ns - nc))[0]
            rows.append(np.stack([ids[a_s], ids[col[a_s]], np.zeros_like(a_s)], 1))
        P = np.concatenate(rows)
        P = P[np.lexsort((P[:, 1], P[:, 0]))]
        cnt_nc = np.empty_like(nc)
        cnt_ns = np.empty_like(ns)
        cnt_nc[ids] = nc
        cnt_ns[ids] = ns
        return P, cnt_nc, cnt_ns


def oracle_pairs(lists, gath):
    rows = [np.stack([np.full(l.size, a), l, g.astype(np.int64)], 1)
            for a, (l, g) in enumerate(zip(lists, gath))]
    P = np.concatenate(rows)
    return P[np.lexsort((P[:, 1], P[:, 0]))]


def rel_err(g, o, scale=None):
    """max |g - o| / max(max |o|, max scale): the scaled criterion for fields that
    may cancel to ~0 (the scale is the per-particle sum of |pair terms|)."""
    g, o = np.asarray(g), np.asarray(o)
    den = np.max(np.abs(o))
    if scale is not None:
        den = max(den, np.max(np.abs(scale)))
    return float(np.max(np.abs(g - o)) / den) if den > 0 else float(np.max(np.abs(g - o)))
