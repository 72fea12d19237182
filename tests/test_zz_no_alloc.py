"""The allocation-free entry point mfmg_divergence_rms_noalloc (partial sums
in the library's fixed device array, result in device memory, no
allocation, copy or wait) against mfmg_divergence_rms on the same inputs:
two calls in a row, the second on a smaller hierarchy, so that the array
keeps the first call's partial sums where the second writes fewer."""

import numpy as np
import pytest

import problems

pytestmark = pytest.mark.gpu


def _tank(l0, obstacle):
    import torch
    from paper_2604_18886_amd import mfmg
    spec = problems.tank_spec(l0, obstacle)
    bc, theta = problems.tank_bc()
    tree = mfmg.build_octree(spec)
    lev, ijk = tree.leaves()
    owner, fdir, other, kind = tree.faces()
    beta = problems.tank_beta(obstacle, lev[owner], ijk[owner], fdir)
    u = problems.tank_velocity(fdir, kind, bc)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                    device="cuda")
    beta_d = dev(beta)
    co = mfmg.assemble_coeffs(tree, beta_d, bc, theta)
    h = mfmg.build_hierarchy(co)
    return h, co, tree, beta_d, dev(u), lev


def test_noalloc_rms_matches_the_allocating_entry_point():
    import torch
    from paper_2604_18886_amd import mfmg
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(77)
    for l0, obstacle in ((6, "sphere"), (3, "star")):
        h, co, tree, beta, u, lev = _tank(l0, obstacle)
        div = mfmg.divergence(h, beta, u)
        noise = torch.as_tensor(rng.uniform(-1.0, 1.0, tree.n_leaves), device="cuda")
        for x in (div, div + 1e-3 * noise):
            want = mfmg.divergence_rms(h, x)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            mfmg.divergence_rms_noalloc(h, x, out)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            got = out.item()
            print(f"  root 1/{2 ** l0} {obstacle}, {tree.n_leaves} leaves: "
                  f"{got:.17e} vs {want:.17e}", flush=True)
            # the same partial sums added in the same order
            assert got == want
            assert free1 == free0
        del h, co, tree
