"""The octree built on the device (the rebuild path of a changing octree):
leaves and faces bit-exact against the oracle octree and the host build,
identical solves and adjoint solves on the device-built tables, device
outputs of a host-built octree, and a sequence of rebuilds around a moving
sphere."""

import numpy as np
import pytest

import problems
from gpu_fixtures import Case, rel
from oracle import discretize as D
from oracle import octree as O

pytestmark = pytest.mark.gpu


def _deep(lmin, lmax, radius, center=(0.31, 0.62, 0.47), band=0.0):
    return {"min_level": lmin, "max_level": lmax, "node_size": 4,
            "prims": [problems.sphere_prim(center, radius, band)]}


SPECS = {
    "single_brick": problems.uniform_spec(2),
    "uniform32": problems.config_spec(1),
    "sphere_band_3_6": problems.config_spec(2, 3, 6),
    "cut_sphere_4_7": problems.config_spec(3, 4, 7),
    "spheres_and_box_4_7": problems.config_spec(4, 4, 7),
    "graded_2_9": _deep(2, 9, 0.05),
    "graded_3_11": _deep(3, 11, 0.004),
    "all_refined_3_5": _deep(3, 5, 0.3, center=(0.5, 0.5, 0.5), band=0.4),
}
ORACLE = {"single_brick", "uniform32", "sphere_band_3_6", "cut_sphere_4_7",
          "spheres_and_box_4_7", "graded_2_9"}


def _equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("name", list(SPECS))
def test_device_octree_matches_host_and_oracle(name):
    import torch
    from paper_2604_18886_amd import mfmg
    spec = SPECS[name]
    th = mfmg.build_octree(spec)
    td = mfmg.build_octree(spec, device=True)
    print(f"\n  {name}: {th.n_leaves} leaves, {th.n_faces} faces", flush=True)
    assert (td.n_leaves, td.n_faces, td.n_leaf_bricks) == (th.n_leaves, th.n_faces,
                                                           th.n_leaf_bricks)
    leaves = th.leaves()
    faces = th.faces()
    assert _equal(td.leaves(), leaves)
    assert _equal(td.faces(), faces)
    ld = [t.cpu().numpy() for t in td.leaves_device()]
    fd = [t.cpu().numpy() for t in td.faces_device()]
    torch.cuda.synchronize()
    assert _equal(ld, leaves)
    assert _equal(fd, faces)
    if name in ORACLE:
        T = O.Octree(spec)
        assert np.array_equal(leaves[0], T.level)
        assert np.array_equal(leaves[1], T.ijk)
        disc = D.Discretization(T, None, (0,) * 6, 0.5)
        assert np.array_equal(faces[0], disc.face_owner)
        assert np.array_equal(faces[1], disc.face_dir)
        assert np.array_equal(faces[2], disc.face_other)
        assert np.array_equal(faces[3], disc.face_kind)


def test_device_outputs_of_a_host_built_octree():
    from paper_2604_18886_amd import mfmg
    th = mfmg.build_octree(SPECS["spheres_and_box_4_7"])
    ld = [t.cpu().numpy() for t in th.leaves_device()]
    fd = [t.cpu().numpy() for t in th.faces_device()]
    assert _equal(ld, th.leaves())
    assert _equal(fd, th.faces())


def test_device_octree_rejects_bad_specs():
    from paper_2604_18886_amd import mfmg
    with pytest.raises(mfmg.MFMGError):
        mfmg.build_octree({"min_level": 5, "max_level": 4, "prims": []}, device=True)
    with pytest.raises(mfmg.MFMGError):
        mfmg.build_octree({"min_level": 3, "max_level": 13, "prims": []}, device=True)
    with pytest.raises(mfmg.MFMGError):
        mfmg.build_octree({"min_level": 3, "max_level": 4, "node_size": 8, "prims": []},
                          device=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_solves_on_device_tables_are_identical(precision):
    """Same tables, same kernels: forward and adjoint solves on the
    device-built octree equal those on the host-built one bit for bit."""
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 5, 7))
    td = mfmg.build_octree(case.spec, device=True)
    sols = []
    for tree in (case.tree, td):
        co = mfmg.assemble_coeffs(tree, case.device(case.beta), case.bc, case.theta)
        h = mfmg.build_hierarchy(co, coarsest_level=3, precision=precision)
        p, st = mfmg.pcg_solve(h, case.device(case.rhs), rtol=1e-10)
        g = case.device(np.where(case.disc.active, p.cpu().numpy() - 1.0, 0.0))
        lam, grad, st2 = mfmg.pcg_solve_adjoint(h, p, g, rtol=1e-10)
        sols.append((p.cpu().numpy(), lam.cpu().numpy(), grad.cpu().numpy(), st["iters"],
                     st2["iters"]))
    a, b = sols
    assert a[3] == b[3] and a[4] == b[4]
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_level_accessors_on_device_tables():
    """Per-level bricks and Algorithm 3 coefficients read back from a
    hierarchy on the device-built octree equal those of the host-built one
    (which the parity tests pin to the oracle)."""
    from paper_2604_18886_amd import mfmg
    case = Case(3, problems.config_spec(3, 4, 6))
    td = mfmg.build_octree(case.spec, device=True)
    hs = []
    for tree in (case.tree, td):
        co = mfmg.assemble_coeffs(tree, case.device(case.beta), case.bc, case.theta)
        hs.append(mfmg.build_hierarchy(co, coarsest_level=3))
    for level in range(3, 7):
        ch, lh = hs[0].level_bricks(level)
        cd, ld = hs[1].level_bricks(level)
        assert np.array_equal(ch, cd) and np.array_equal(lh, ld)
        assert np.array_equal(hs[0].level_coeffs(level).cpu().numpy(),
                              hs[1].level_coeffs(level).cpu().numpy())


def test_rebuilds_around_a_moving_sphere():
    """Time loop: each step rebuilds the octree on the device around the
    sphere's new position, re-assembles, re-coarsens and solves; the
    topology matches the oracle octree and the solution the oracle's
    operator at every step."""
    from paper_2604_18886_amd import mfmg
    bc = (0, 0, 0, 1, 0, 0)
    for step in range(4):
        c = (0.35 + 0.07 * step, 0.5, 0.45 + 0.03 * step)
        spec = _deep(4, 7, 0.15, center=c, band=0.02)
        td = mfmg.build_octree(spec, device=True)
        T = O.Octree(spec)
        lev, ijk = td.leaves()
        assert np.array_equal(lev, T.level) and np.array_equal(ijk, T.ijk)
        disc = D.Discretization(T, None, bc, 0.5)
        owner, fdir, other, kind = td.faces()
        assert np.array_equal(owner, disc.face_owner)
        assert np.array_equal(fdir, disc.face_dir)
        assert np.array_equal(other, disc.face_other)
        assert np.array_equal(kind, disc.face_kind)
        beta = np.ones(td.n_faces)
        disc.set_beta(beta)
        rhs = problems.rhs_random(3, lev, ijk)
        import torch
        dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
        co = mfmg.assemble_coeffs(td, dev(beta), bc, 0.5)
        h = mfmg.build_hierarchy(co, coarsest_level=3, precision=mfmg.MIXED)
        p, st = mfmg.pcg_solve(h, dev(rhs), rtol=1e-10)
        x = p.cpu().numpy()
        act = disc.active
        r = np.where(act, rhs - disc.A @ x, 0.0)
        res = np.linalg.norm(r) / np.linalg.norm(np.where(act, rhs, 0.0))
        print(f"  step {step}: {td.n_leaves} leaves, {st['iters']} iterations, "
              f"oracle-measured residual {res:.2e}", flush=True)
        assert st["status"] == 0 and res <= 1e-10 * (1 + 1e-4)
