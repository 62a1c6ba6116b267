"""query_hoph_noalloc: the query path on the library's fixed per-device
scratch.  Through the C ABI, two calls in a row (the second with fewer
queries, so stale scratch contents from the first must not leak into it) give
exactly query_hoph's CSR output, which is the oracle's; sizes beyond the
scratch are refused before any launch."""
from fractions import Fraction

import numpy as np
import pytest

import paper_1805_11254_amd as H
from oracle import scale
import workloads as W
from tests.hoph_testutil import dev_csr, oracle_sketch, params_of, to_u32

pytestmark = pytest.mark.gpu


def _lists(o, i):
    o = o.cpu().numpy()
    i = to_u32(i)
    return [i[o[j]:o[j + 1]].tolist() for j in range(len(o) - 1)]


def test_noalloc_query_equals_query_hoph_and_oracle():
    import torch
    print("[case] query_hoph_noalloc, two calls", flush=True)
    w = W.hoph_bovw(n=20_011, n_q=64, seed=61, planted_frac=0.03)
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    qids, qoffs = dev_csr(w.queries)
    sig = H.sketch_oph(p, ids, offs)
    qsig = H.sketch_oph(p, qids, qoffs)
    idx = H.Index(p, sig)
    osig, oq = oracle_sketch(w, w.collection), oracle_sketch(w, w.queries)
    assert (to_u32(sig) == osig).all() and (to_u32(qsig) == oq).all()
    for rows in (list(range(64)), [3, 17, 18, 40, 41, 42, 50, 62, 63]):
        q = qsig[rows].contiguous()
        got = _lists(*H.query_hoph_noalloc(idx, q, T=w.T, eps=w.eps))
        want = _lists(*H.query_hoph(idx, q, T=w.T, eps=w.eps))
        oo, oi, _ = scale.query(osig, oq[rows], goph=False, kp=w.kp, T=Fraction(*w.T), eps=Fraction(*w.eps),
                                ra=w.ra, rb=w.rb)
        assert got == want, len(rows)
        assert got == [oi[oo[j]:oo[j + 1]].tolist() for j in range(len(rows))], len(rows)
        assert sum(len(x) for x in got) > 0
    # an explicit output buffer that is too small: the pairs needed are reported
    with pytest.raises(H.HophError) as ei:
        H.query_hoph_noalloc(idx, qsig, T=w.T, eps=w.eps, capacity=1)
    assert ei.value.status == H.HOPH_E_CAPACITY and ei.value.needed > 1
    # more queries than the scratch takes: refused before any launch
    big = torch.zeros((4097, w.k), dtype=torch.int32, device="cuda")
    with pytest.raises(H.HophError) as ei:
        H.query_hoph_noalloc(idx, big, T=w.T, eps=w.eps)
    assert ei.value.status == H.HOPH_E_CAPACITY
    # the entry point still answers after the refusals
    assert _lists(*H.query_hoph_noalloc(idx, qsig[:5].contiguous(), T=w.T, eps=w.eps)) == \
        _lists(*H.query_hoph(idx, qsig[:5].contiguous(), T=w.T, eps=w.eps))
    idx.free()
