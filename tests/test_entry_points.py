"""CPU checks of the entry points around the library: the benchmark refuses
more than one GPU, and the binding fails loudly when the library is absent
(there is no CPU fallback)."""
import os
import subprocess
import sys

import pytest

from paper_2309_16724_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_missing_library_raises(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        B.load(str(tmp_path / "libdmrg_hpsi.so"))


def test_davidson_defaults_match_the_oracle():
    """The device-versus-oracle Davidson tests run both sides with their
    defaults: the preconditioner floor, tolerance and subspace size must
    agree (reading of the Davidson details, relative floor 1e-2)."""
    import inspect
    from oracle.davidson import davidson as odav
    from oracle import mlp as omlp
    from paper_2309_16724_amd.hpsi import Plan
    lib = inspect.signature(Plan.davidson).parameters
    ref = inspect.signature(odav).parameters
    for k in ("floor", "tol", "m_max", "max_iter"):
        assert lib[k].default == ref[k].default, k
    col = inspect.signature(Plan.collect).parameters
    assert col["floor"].default == ref["floor"].default
    for f in (omlp.diagonal_step, omlp.training_rows, omlp.mlp_step):
        assert inspect.signature(f).parameters["floor"].default == ref["floor"].default


def test_bench_layout_matches_the_documented_order():
    """bench.py computes wavefunction block offsets itself (its timed legs do
    not touch the oracle); they follow the order the header fixes."""
    import bench
    from oracle.layout import psi_blocks
    from paper_2309_16724_amd.synth.problem import random_problem
    for args in ((12, 12, 0, 3, 64), (11, 11, 1, 4, 48)):
        p = random_problem(*args, p=5)
        assert bench.psi_layout(p.left.sectors, p.right.sectors, p.n_elec, p.two_s) == \
            psi_blocks(p.left.sectors, p.right.sectors, p.n_elec, p.two_s)
