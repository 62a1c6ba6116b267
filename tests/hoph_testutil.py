"""Helpers shared by the GPU tests: moving workloads to the device, running the
library and the oracle on the same inputs, comparing CSR outputs."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import paper_1805_11254_amd as H
from oracle import scale, tiny
import workloads as W


def dev_csr(coll, device="cuda"):
    import torch
    ids = torch.from_numpy(np.ascontiguousarray(coll.ids).view(np.int32)).to(device)
    offs = torch.from_numpy(np.ascontiguousarray(coll.offsets).view(np.int64)).to(device)
    return ids, offs


def params_of(w: W.Workload, device="cuda") -> H.SketchParams:
    import torch
    perm = None
    if w.hash_kind == W.HASH_TABLE:
        perm = torch.from_numpy(w.perm.view(np.int32)).to(device)
    return H.SketchParams(w.layout, w.k, w.kp, w.hash_kind, w.universe, w.ra, w.rb, w.ha, w.hb, perm)


def oracle_sketch(w: W.Workload, coll, which=None, allow_empty=False):
    return scale.sketch(coll.ids, coll.offsets, hash_kind=w.hash_kind, universe=w.universe, layout=w.layout,
                        k=w.k, kp=w.kp, ra=w.ra, rb=w.rb, ha=w.ha, hb=w.hb, perm=w.perm, which=which,
                        allow_empty=allow_empty)


def gpu_sketch(w: W.Workload, coll, params=None):
    ids, offs = dev_csr(coll)
    p = params or params_of(w)
    return H.sketch_oph(p, ids, offs)


def to_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def csr_lists(offsets, ids):
    offsets = np.asarray(offsets).astype(np.int64)
    ids = np.asarray(ids)
    return [ids[offsets[i]:offsets[i + 1]].tolist() for i in range(len(offsets) - 1)]


def gpu_query(kind, index, qsigs, T, eps, policy, **kw):
    fn = {"goph": H.query_goph, "hoph": H.query_hoph}[kind]
    offs, ids = fn(index, qsigs, T=T, eps=eps, policy=policy, **kw)
    return offs.cpu().numpy(), to_u32(ids)


def oracle_query(w: W.Workload, sigs, qsigs, T, eps, policy):
    offs, ids, steps = scale.query(sigs, qsigs, goph=w.goph, kp=w.kp, T=Fraction(*T), eps=Fraction(*eps),
                                   policy=policy, ra=w.ra, rb=w.rb)
    return offs, ids
