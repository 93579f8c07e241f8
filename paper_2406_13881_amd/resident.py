"""Resident batches: CFGs packed into a few device tensors owned by torch.

Torch only provides device memory and streams here; every step of the solve
runs in libompd's kernels.  Arrays of one kind (successor CSR, edge kinds,
spaces, read/write bitmaps, each output) are packed back to back into one
tensor, and each CFG's descriptor points into them, so a batch of thousands
of CFGs costs a handful of allocations and host-to-device copies.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from . import OUTPUTS, Context, DeviceCFG, DeviceResult, Plan

_U64 = "int64"   # torch has no uint64; the bits are the same


def _offsets(sizes: Sequence[int]) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(np.asarray(sizes, dtype=np.int64), out=off[1:])
    return off


class ResidentBatch:
    """Upload ``cfgs`` once, allocate every requested output on the device,
    and build an ``ompd`` plan over them."""

    def __init__(self, ctx: Context, cfgs: Sequence, want: Sequence[str] = OUTPUTS, flags: int = 0,
                 device: str = "cuda", with_boundaries: bool = True):
        import torch
        self.torch = torch
        self.n = len(cfgs)
        self.want = tuple(want)
        nb = np.array([c.n_blocks for c in cfgs], dtype=np.int64)
        ne = np.array([np.asarray(c.succ_idx).shape[0] for c in cfgs], dtype=np.int64)
        nv = np.array([c.n_vars for c in cfgs], dtype=np.int64)
        wd = (nv + 63) // 64
        self.nb, self.ne, self.nv, self.wd = nb, ne, nv, wd
        self.o_ptr = _offsets(nb + 1)
        self.o_edge = _offsets(ne)
        self.o_blk = _offsets(nb)
        self.o_bw = _offsets(nb * wd)
        self.o_ew = _offsets(ne * wd)
        self.o_var = _offsets(nv)
        self.o_w = _offsets(wd)

        def cat(parts, dtype):
            parts = [np.ascontiguousarray(p, dtype=dtype).reshape(-1) for p in parts]
            return np.concatenate(parts) if parts else np.zeros(0, dtype)

        dev = torch.device(device)
        t = lambda a: torch.from_numpy(a).to(dev)
        self.d_sp = t(cat([c.succ_ptr for c in cfgs], np.int32))
        self.d_si = t(cat([c.succ_idx for c in cfgs], np.int32))
        self.d_kd = t(cat([c.edge_kind for c in cfgs], np.uint8))
        self.d_spc = t(cat([c.space for c in cfgs], np.uint8))
        self.d_R = t(cat([c.R for c in cfgs], np.uint64).view(np.int64))
        self.d_W = t(cat([c.W for c in cfgs], np.uint64).view(np.int64))
        bnd = {}
        if with_boundaries:
            for name in ("entry_valid_h", "entry_valid_d", "exit_live_h", "exit_live_d"):
                vals = [getattr(c, name, None) for c in cfgs]
                if any(v is not None for v in vals):
                    full = []
                    for c, v in zip(cfgs, vals):
                        if v is None:
                            v = c.boundary()[("entry_valid_h", "entry_valid_d", "exit_live_h", "exit_live_d").index(name)]
                        full.append(np.asarray(v, dtype=np.uint64))
                    bnd[name] = t(cat(full, np.uint64).view(np.int64))
        self.d_bnd = bnd
        # scalar marks (firstprivate candidates), zero words for CFGs without marks
        self.d_sc = None
        if any(getattr(c, "scalar", None) is not None for c in cfgs):
            marks = [np.zeros(int(w), np.uint64) if getattr(c, "scalar", None) is None else c.scalar
                     for c, w in zip(cfgs, wd)]
            self.d_sc = t(cat(marks, np.uint64).view(np.int64))
        total = {"bw": int(self.o_bw[-1]), "ew": int(self.o_ew[-1]), "var": int(self.o_var[-1]), "blk": int(self.o_blk[-1])}
        self.out = {}
        for k in self.want:
            if k.startswith("ins_edge"):
                self.out[k] = torch.zeros(max(total["ew"], 1), dtype=torch.int64, device=dev)
            elif k == "var_kind":
                self.out[k] = torch.zeros(max(total["var"], 1), dtype=torch.uint8, device=dev)
            elif k in ("after_dev", "before_dev"):
                self.out[k] = torch.zeros(max(total["blk"], 1), dtype=torch.uint8, device=dev)
            else:
                self.out[k] = torch.zeros(max(total["bw"], 1), dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        self.dcfgs: List[DeviceCFG] = []
        self.dres: List[DeviceResult] = []
        for i, c in enumerate(cfgs):
            g = DeviceCFG(n_blocks=int(nb[i]), n_edges=int(ne[i]), n_vars=int(nv[i]), entry=int(c.entry),
                          exit=int(c.exit),
                          succ_ptr=self.d_sp.data_ptr() + 4 * int(self.o_ptr[i]),
                          succ_idx=self.d_si.data_ptr() + 4 * int(self.o_edge[i]),
                          edge_kind=self.d_kd.data_ptr() + int(self.o_edge[i]),
                          space=self.d_spc.data_ptr() + int(self.o_blk[i]),
                          read_bits=self.d_R.data_ptr() + 8 * int(self.o_bw[i]),
                          write_bits=self.d_W.data_ptr() + 8 * int(self.o_bw[i]))
            for name, field in (("entry_valid_h", "entry_valid_host"), ("entry_valid_d", "entry_valid_dev"),
                                ("exit_live_h", "exit_live_host"), ("exit_live_d", "exit_live_dev")):
                if name in bnd:
                    setattr(g, field, bnd[name].data_ptr() + 8 * int(self.o_w[i]))
            if self.d_sc is not None and getattr(c, "scalar", None) is not None:
                g.scalar = self.d_sc.data_ptr() + 8 * int(self.o_w[i])
            self.dcfgs.append(g)
            r = DeviceResult()
            for k in self.want:
                base = self.out[k].data_ptr()
                if k.startswith("ins_edge"):
                    setattr(r, k, base + 8 * int(self.o_ew[i]))
                elif k == "var_kind":
                    setattr(r, k, base + int(self.o_var[i]))
                elif k in ("after_dev", "before_dev"):
                    setattr(r, k, base + int(self.o_blk[i]))
                else:
                    setattr(r, k, base + 8 * int(self.o_bw[i]))
            self.dres.append(r)
        self.plan = Plan(ctx, self.dcfgs, self.dres, flags)

    def facts(self) -> int:
        return int(((self.nb - 2) * self.nv).sum())

    def run(self, stream: int = 0):
        self.plan.run(stream)

    def fetch(self, i: int) -> Dict[str, np.ndarray]:
        """Copy CFG i's outputs to host numpy arrays (shapes as the oracle's)."""
        out = {}
        nb, ne, nv, wd = int(self.nb[i]), int(self.ne[i]), int(self.nv[i]), int(self.wd[i])
        for k in self.want:
            t = self.out[k]
            if k.startswith("ins_edge"):
                a = t[int(self.o_ew[i]):int(self.o_ew[i + 1])].cpu().numpy().view(np.uint64).reshape(ne, wd)
            elif k == "var_kind":
                a = t[int(self.o_var[i]):int(self.o_var[i + 1])].cpu().numpy()
            elif k in ("after_dev", "before_dev"):
                a = t[int(self.o_blk[i]):int(self.o_blk[i + 1])].cpu().numpy()
            else:
                a = t[int(self.o_bw[i]):int(self.o_bw[i + 1])].cpu().numpy().view(np.uint64).reshape(nb, wd)
            out[k] = a
        return out

    def fetch_all(self):
        """Copy every output of the batch to the host at once (one copy per output) and
        return a function i -> CFG i's outputs (views, shapes as fetch(i))."""
        host = {k: self.out[k].cpu().numpy() for k in self.want}
        nb, ne, nv, wd = self.nb, self.ne, self.nv, self.wd

        def get(i: int) -> Dict[str, np.ndarray]:
            out = {}
            for k in self.want:
                a = host[k]
                if k.startswith("ins_edge"):
                    out[k] = a[int(self.o_ew[i]):int(self.o_ew[i + 1])].view(np.uint64).reshape(int(ne[i]), int(wd[i]))
                elif k == "var_kind":
                    out[k] = a[int(self.o_var[i]):int(self.o_var[i + 1])]
                elif k in ("after_dev", "before_dev"):
                    out[k] = a[int(self.o_blk[i]):int(self.o_blk[i + 1])]
                else:
                    out[k] = a[int(self.o_bw[i]):int(self.o_bw[i + 1])].view(np.uint64).reshape(int(nb[i]), int(wd[i]))
            return out
        return get

    def close(self):
        if getattr(self, "plan", None) is not None:
            self.plan.close()
            self.plan = None
