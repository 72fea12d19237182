"""CPU tests of the C-ABI library: it loads, exports every symbol that
include/mfmg.h declares, and its host-only octree calls reproduce the
oracle's topology bit for bit (no device call is made here)."""

import os
import re

import numpy as np
import pytest

import problems
from oracle import discretize as D
from oracle import octree as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mfmg.h")).read()
    return sorted(set(re.findall(r"\b(mfmg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2604_18886_amd import mfmg
    lib = mfmg.load_library()
    names = declared_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
        assert n in mfmg.SIGNATURES, n


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_library_topology_matches_oracle(cfg):
    from paper_2604_18886_amd import mfmg
    spec = problems.config_spec(cfg)
    tree = mfmg.build_octree(spec)
    T = O.Octree(spec)
    lev, ijk = tree.leaves()
    assert np.array_equal(lev, T.level) and np.array_equal(ijk, T.ijk)
    owner, d, other, kind = tree.faces()
    disc = D.Discretization(T, None, *problems.config_bc(cfg))
    assert np.array_equal(owner, disc.face_owner)
    assert np.array_equal(d, disc.face_dir)
    assert np.array_equal(other, disc.face_other)
    assert np.array_equal(kind, disc.face_kind)


def test_library_topology_large_workload_leaves():
    from paper_2604_18886_amd import mfmg
    spec = problems.config_spec(4)
    tree = mfmg.build_octree(spec)
    T = O.Octree(spec)
    lev, ijk = tree.leaves()
    assert tree.n_leaves == T.n
    assert np.array_equal(lev, T.level) and np.array_equal(ijk, T.ijk)


def test_invalid_arguments_return_status():
    from paper_2604_18886_amd import mfmg
    with pytest.raises(mfmg.MFMGError) as e:
        mfmg.build_octree({"min_level": 1, "max_level": 3, "node_size": 4, "prims": []})
    assert e.value.status == -1
    with pytest.raises(mfmg.MFMGError):
        mfmg.build_octree({"min_level": 3, "max_level": 3, "node_size": 8, "prims": []})
    with pytest.raises(mfmg.MFMGError):
        mfmg.build_octree({"min_level": 3, "max_level": 4, "node_size": 4,
                           "prims": [{"kind": 7}]})


def test_binding_rejects_wrong_vector_lengths():
    """The C ABI cannot check the length of a device buffer: the binding
    rejects a vector of the wrong length or type before any library call."""
    import torch
    from paper_2604_18886_amd import mfmg

    class _Fake:  # stands in for a hierarchy: sizes only, never reaches the library
        _h = None
        n_leaves = 64

        class coeffs:
            class tree:
                n_faces = 240

    mfmg.load_library()
    h = _Fake()
    for bad in (torch.zeros(63, dtype=torch.float64), torch.zeros(64, dtype=torch.float32)):
        with pytest.raises(ValueError):
            mfmg.pcg_solve(h, bad)
        with pytest.raises(ValueError):
            mfmg.apply_operator(h, bad)
        with pytest.raises(ValueError):
            mfmg.divergence_rms(h, bad)
    with pytest.raises(ValueError):
        mfmg.divergence(h, torch.zeros(239, dtype=torch.float64),
                        torch.zeros(240, dtype=torch.float64))
