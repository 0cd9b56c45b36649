"""Repeatability of a full-size launch: the same batch propagated twice must give the
same state bit for bit and the same Arnoldi iteration counts.  Cross-wave hazards in the
workgroup's shared memory (a coefficient overwritten before every wave has read it)
show up here as run-to-run differences long before they move a sampled packet past
the parity bound.  Packets of N = 2048 with momenta of up to 5 a.u. need 8-11 Arnoldi
iterations per Suzuki order-6 substep of 10 a.u., mostly without a second
Gram-Schmidt pass."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1902_04661_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_large_batch_is_repeatable_and_matches_oracle():
    from paper_1902_04661_amd import gqd
    gqd.load_library()
    items = I.ragged_batch(768, seed=0, fixed_n=2048)
    prop = gqd.from_items(items)
    opts = dict(tol=1e-14, restart=32)
    psi0 = prop.pack([it.psi0 for it in items])
    outs, stats = [], []
    for _ in range(3):
        psi = psi0.clone()
        st = prop.propagate(psi, "midp", "suzuki", 6, 10.0, 1, gqd.SolverOpts(**opts))
        outs.append(psi)
        stats.append((st.iterations, st.h_applies, st.max_iters))
        print(f"iterations {st.iterations}, per solve {st.iterations / st.solves:.3f}, "
              f"max {st.max_iters}", flush=True)
    for k in (1, 2):
        ndiff = int((outs[k] != outs[0]).sum())
        print(f"run {k}: {ndiff} differing elements", flush=True)
        assert ndiff == 0 and stats[k] == stats[0]
    got = prop.unpack(outs[0])
    for b in (0, 383, 767):
        ref = O.propagate(O.model_from_item(items[b]), items[b].psi0, O.MIDP, O.SUZUKI, 6, 10.0, 1,
                          O.SolverOpts(**opts))
        r = float(np.linalg.norm(got[b] - ref) / np.linalg.norm(ref))
        print(f"packet {b}: rel {r:.2e}", flush=True)
        assert r <= 1e-12
