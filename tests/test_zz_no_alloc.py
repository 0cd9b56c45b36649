"""The allocation-free propagation (gqd_propagate_noalloc, the library's static device
scratch instead of the caller's workspace) against gqd_propagate on the same inputs: two
calls in a row, the second on a smaller batch, each bit-identical to the workspace path
(same kernels and arithmetic, only the workspace address and the launch order of the
size classes differ)."""
import numpy as np
import pytest
import torch

from paper_1902_04661_amd import inputs as I

pytestmark = pytest.mark.gpu


def batch(sizes, seed):
    rng = np.random.default_rng(seed)
    return [I.nai_like_item(n, q0=float(rng.uniform(4.5, 6)), p0=float(rng.uniform(-5, 5)),
                            amp=float(rng.uniform(0.1, 0.8))) for n in sizes]


@pytest.mark.parametrize("sizes,seed", [((2048, 512, 4096, 256), 21), ((1024,), 22)])
def test_noalloc_matches_workspace_path_twice(sizes, seed):
    from paper_1902_04661_amd import gqd
    gqd.load_library()
    items = batch(sizes, seed)
    opts = gqd.SolverOpts(tol=1e-14, restart=32)
    with gqd.from_items(items) as ref_prop, gqd.from_items(items) as prop:
        ref = ref_prop.pack([it.psi0 for it in items])
        st_ref = ref_prop.propagate(ref, "midp", "suzuki", 4, 10.0, 2, opts)
        for call in range(2):
            psi = prop.pack([it.psi0 for it in items])
            st = prop.propagate_noalloc(psi, "midp", "suzuki", 4, 10.0, 2, opts)
            print(f"sizes {sizes} call {call}: max |diff| {float((psi - ref).abs().max()):.1e}, "
                  f"iterations {st.iterations} vs {st_ref.iterations}", flush=True)
            assert torch.equal(psi, ref)
            assert st.iterations == st_ref.iterations and st.solves == st_ref.solves


def test_noalloc_rejects_what_does_not_fit():
    from paper_1902_04661_amd import gqd
    gqd.load_library()
    items = batch((4096,) * 16, 23)  # 16 x (32 + 6) x 2 x 4096 x 16 B = 80 MB > 64 MiB at restart 32
    with gqd.from_items(items) as prop:
        psi = prop.pack([it.psi0 for it in items])
        with pytest.raises(gqd.GqdError, match="static scratch"):
            prop.propagate_noalloc(psi, "midp", "suzuki", 2, 10.0, 1, gqd.SolverOpts(restart=32))
        # the state is untouched by the rejected call
        assert torch.equal(psi, prop.pack([it.psi0 for it in items]))
