"""The allocation-free search (hjb_policy_sweep_noalloc) against hjb_policy_sweep through the C ABI.

Its scratch is one static device array per GPU shared by every call, so the test runs two calls in a row,
the second on a smaller grid (a different handle) after the first has left its values in the array, and
compares each with the allocating entry point's outputs bit for bit: policies, minima, margins, tie counts,
changed counts and tau.  Calls that leave out the read-back only enqueue work; their outputs must agree too.
A grid beyond the scratch limit and a scale s the tables were not built for are rejected.
"""
import numpy as np
import pytest

import workloads
from gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _outputs(slhjb, solver, inst, fn, seed, theta, read_back=True):
    X, U = workloads.random_fields(inst, seed=seed)
    a_in = workloads.random_policy(inst, seed=seed + 1)
    dev = "cuda"
    a_out = torch.full((inst.N,), 7, dtype=torch.int16, device=dev)
    gmin = torch.full((inst.N,), -3.0, dtype=torch.float64, device=dev)
    margin = torch.full((inst.N,), -3.0, dtype=torch.float64, device=dev)
    ties = torch.full((inst.N,), -3, dtype=torch.int32, device=dev)
    kw = {} if fn == "policy_sweep" else dict(read_back=read_back)
    nch, tau = getattr(solver, fn)(to_dev(X), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), 0.3, 1.0 / 64, theta, 1.0,
                                   to_dev(a_in), a_out, gmin, margin, ties, **kw)
    torch.cuda.synchronize()
    return dict(alpha=to_np(a_out), gmin=to_np(gmin), margin=to_np(margin), ties=to_np(ties), nch=nch, tau=tau)


def _compare(a, b, with_counts=True):
    for k in ("alpha", "gmin", "margin", "ties"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    if with_counts:
        assert a["nch"] == b["nch"] and a["tau"] == b["tau"]


def test_noalloc_search_matches_allocating_entry_point(slhjb):
    big = workloads.config_c2(257)
    small = workloads.config_c2(65)
    for rnd, (inst, theta) in enumerate(((big, 0.5), (small, 1.0), (big, 1.0))):
        solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
        ref = _outputs(slhjb, solver, inst, "policy_sweep", 10 + rnd, theta)
        got = _outputs(slhjb, solver, inst, "policy_sweep_noalloc", 10 + rnd, theta)
        log(f"call {rnd}: {inst.name} theta={theta}: changed {got['nch']} / {ref['nch']}, tau {got['tau']:.6e}")
        _compare(got, ref)
        quiet = _outputs(slhjb, solver, inst, "policy_sweep_noalloc", 10 + rnd, theta, read_back=False)
        _compare(quiet, ref, with_counts=False)
        solver.close()


def test_noalloc_search_3d_and_ragged(slhjb):
    rng_inst = workloads.config_c5(17, n_steps=1)
    solver = slhjb.Solver.from_instance(rng_inst, slhjb.Options(precision=1))
    ref = _outputs(slhjb, solver, rng_inst, "policy_sweep", 3, 1.0)
    got = _outputs(slhjb, solver, rng_inst, "policy_sweep_noalloc", 3, 1.0)
    _compare(got, ref)
    solver.close()


def test_noalloc_search_rejections(slhjb):
    inst = workloads.config_c2(65)
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=1))
    X, U = workloads.random_fields(inst, seed=5)
    a = to_dev(workloads.random_policy(inst, seed=6))
    out = torch.empty_like(a)
    args = (to_dev(X), to_dev(U), to_dev(inst.f0), to_dev(inst.f1), 0.0, 0.01, 1.0)
    with pytest.raises(slhjb.HJBError):
        solver.policy_sweep_noalloc(*args, 1.25, a, out)   # tables are built for s = 1
    solver.policy_sweep(*args, 1.25, a, out)               # builds them for 1.25
    solver.policy_sweep_noalloc(*args, 1.25, a, out)
    solver.close()
    # a grid whose tiles need more than the 1 MiB scratch (about 43,000 tiles)
    n = 3401
    big = slhjb.Solver(2, (n, n), (0.0, 0.0), 1.0 / (n - 1), np.array([[[1.0, 0.0]]]),
                       options=slhjb.Options(precision=1, precond=slhjb.PRECOND_JACOBI, restart=2))
    z = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    a0 = torch.zeros(n * n, dtype=torch.int16, device="cuda")
    with pytest.raises(slhjb.HJBError, match="scratch"):
        big.policy_sweep_noalloc(z, z, z, z, 0.0, 0.01, 1.0, 1.0, a0, torch.empty_like(a0))
    big.close()
