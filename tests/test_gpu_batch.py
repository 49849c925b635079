"""Batched solves (hjb_setup_batch / hjb_solve_batch) against the oracle and against single-instance solves.

Each batch mixes grid sizes, coefficient models, control counts and multigrid depths: x-scaled
two-asset instances, ragged boxes with discounting and drift, a grid that cannot coarsen (solved on
one level in LDS) and one that cannot coarsen and is too large for that (Jacobi sweeps).  All
instances share one schedule.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import log, to_dev, to_np
from policy_parity import check_march_policies

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _toy(n, K, P, seed, c=True, drift=True):
    rng = np.random.default_rng(seed)
    dim = len(n)
    N = int(np.prod(n))
    inst = workloads.Instance(name=f"toy{n}", dim=dim, n=tuple(n), lo=(0.0,) * dim, h=1.0 / (max(n) - 1), K=K, P=P,
                              sigma=rng.normal(size=(K, P, dim)),
                              drift=rng.normal(size=(K, dim)) * 0.4 if drift else None,
                              c=-rng.uniform(0.0, 1.0, size=K) if c else None, f0=rng.normal(size=N),
                              f1=rng.normal(size=N), g=rng.normal(size=N), psi=np.zeros(N),
                              dts=np.array([0.05]), thetas=np.array([1.0]))
    inst.psi = np.where(inst.boundary_mask(), rng.normal(size=N) * 0.3, 0.0)
    return inst


def _schedule(insts, dts, thetas):
    for inst in insts:
        inst.dts = np.asarray(dts, float)
        inst.thetas = np.asarray(thetas, float)
    return insts


def _batch_2d():
    insts = [workloads.c4_instance(65, 0.12, 0.29, 0.35, 0.02),
             workloads.c4_instance(17, 0.15, 0.31, 0.45, 0.04),
             _toy((37, 29), K=5, P=2, seed=3),
             workloads.c4_instance(33, 0.18, 0.30, 0.32, 0.01),
             _toy((30, 27), K=4, P=1, seed=9),        # odd cell counts: one level, LDS solve
             _toy((52, 47), K=3, P=1, seed=11)]       # one level of 2444 nodes: Jacobi sweeps
    return _schedule(insts, [0.02, 0.02, 0.01, 0.01], [1.0, 1.0, 0.5, 0.5])


def _run_batch(slhjb, insts, opts):
    bt = slhjb.Batch(insts, opts)
    g, psi, f0, f1 = (to_dev(bt.concat(k)) for k in ("g", "psi", "f0", "f1"))
    U = torch.empty_like(g)
    pol = torch.empty((len(insts[0].dts), bt.total), dtype=torch.int16, device="cuda")
    st = bt.solve(g, psi, f0, f1, insts[0].dts, insts[0].thetas, 1.0, U, pol)
    out = [to_np(u) for u in bt.split(U)]
    pols = [to_np(pol[:, o:o + inst.N]) for inst, o in zip(insts, bt.offsets)]
    bt.close()
    return out, pols, st


@pytest.mark.parametrize("precision,max_levels", [(0, 2), (1, 2), (1, 0)], ids=["fp64", "mixed", "mixed-deep"])
def test_batch_matches_oracle_and_single(slhjb, precision, max_levels):
    insts = _batch_2d()
    log(f"batch of {len(insts)} 2D instances, precision={precision}, max_levels={max_levels}")
    opts = slhjb.Options(precision=precision, max_levels=max_levels)
    Ub, pb, st = _run_batch(slhjb, insts, opts)
    for b, inst in enumerate(insts):
        ref = oracle.march(inst, keep_policies=True, keep_values=True)
        rel = np.max(np.abs(Ub[b] - ref["U"])) / np.max(np.abs(ref["U"]))
        check_march_policies(inst, ref, pb[b], log=log)
        solver = slhjb.Solver.from_instance(inst, opts)
        g = to_dev(inst.g)
        U1 = torch.empty_like(g)
        pol1 = torch.empty((len(inst.dts), inst.N), dtype=torch.int16, device="cuda")
        st1 = solver.solve(g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas, 1.0, U1, pol1)
        solver.close()
        rel1 = np.max(np.abs(Ub[b] - to_np(U1))) / np.max(np.abs(to_np(U1)))
        log(f"  {inst.name}: batch pi={st[b].pi_total} krylov={st[b].krylov_total} | single pi={st1.pi_total} "
            f"krylov={st1.krylov_total} | rel vs oracle {rel:.2e}, vs single {rel1:.2e}")
        assert st[b].steps_done == len(inst.dts)
        assert rel <= 1e-10
        assert rel1 <= 1e-10


def test_batch_of_one_equals_single(slhjb):
    inst = _schedule([workloads.c4_instance(65, 0.12, 0.29, 0.35, 0.02)], [0.02] * 3, [1.0] * 3)[0]
    Ub, pb, st = _run_batch(slhjb, [inst], slhjb.Options(precision=0))
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=0))
    g = to_dev(inst.g)
    U1 = torch.empty_like(g)
    pol1 = torch.empty((3, inst.N), dtype=torch.int16, device="cuda")
    solver.solve(g, to_dev(inst.psi), to_dev(inst.f0), to_dev(inst.f1), inst.dts, inst.thetas, 1.0, U1, pol1)
    solver.close()
    np.testing.assert_allclose(Ub[0], to_np(U1), rtol=0, atol=1e-12 * np.max(np.abs(Ub[0])))
    np.testing.assert_array_equal(pb[0], to_np(pol1))


def test_batch_3d(slhjb):
    insts = _schedule([workloads.config_c5(17, n_steps=2), workloads.config_c5(9, K=16, n_steps=2),
                       _toy((11, 9, 13), K=5, P=1, seed=4)], [1.0 / 32] * 2, [1.0, 1.0])
    log("batch of 3D instances")
    Ub, pb, st = _run_batch(slhjb, insts, slhjb.Options(precision=1))
    for b, inst in enumerate(insts):
        ref = oracle.march(inst, keep_policies=True, keep_values=True)
        rel = np.max(np.abs(Ub[b] - ref["U"])) / np.max(np.abs(ref["U"]))
        check_march_policies(inst, ref, pb[b], log=log)
        log(f"  {inst.name}: pi={st[b].pi_total} krylov={st[b].krylov_total} rel {rel:.2e}")
        assert rel <= 1e-10


def test_batch_rejects_bad_options(slhjb):
    insts = _batch_2d()[:2]
    with pytest.raises(slhjb.HJBError):
        slhjb.Batch(insts, slhjb.Options(nu1=2, nu2=1))
    with pytest.raises(slhjb.HJBError):
        slhjb.Batch(insts, slhjb.Options(precond=slhjb.PRECOND_JACOBI))
    with pytest.raises(slhjb.HJBError):
        slhjb.Batch(insts, slhjb.Options(krylov=slhjb.KRYLOV_BICGSTAB))


def test_batch_graph_replays_match_eager(slhjb):
    """Batched restart cycles (m Arnoldi steps with their V-cycles and device-side Givens rotations) and
    V-cycles replayed from captured graphs (reused across restart cycles, policy iterations and time steps,
    with eager work in between) give the eager results bit for bit."""
    insts = _batch_2d()[:4]
    Ug, pg, _ = _run_batch(slhjb, insts, slhjb.Options(precision=1, use_graphs=1))
    Ue, pe, _ = _run_batch(slhjb, insts, slhjb.Options(precision=1, use_graphs=0))
    for a, b, pa, pb_ in zip(Ug, Ue, pg, pe):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(pa, pb_)


def test_batch_mixed_coefficient_models(slhjb):
    """Per-node sigma (Problem A at two sizes), x-scaled and constant coefficients in one batch."""
    insts = _schedule([workloads.problem_a(41), workloads.problem_a(81),
                       workloads.c4_instance(33, 0.15, 0.31, 0.45, 0.04), _toy((37, 29), K=5, P=2, seed=3)],
                      [0.125, 0.125], [1.0, 1.0])
    Ub, pb, st = _run_batch(slhjb, insts, slhjb.Options(precision=1))
    for b, inst in enumerate(insts):
        ref = oracle.march(inst, keep_policies=True, keep_values=True)
        rel = np.max(np.abs(Ub[b] - ref["U"])) / np.max(np.abs(ref["U"]))
        check_march_policies(inst, ref, pb[b], log=log)
        log(f"  {inst.name}: pi={st[b].pi_total} krylov={st[b].krylov_total} rel {rel:.2e}")
        assert rel <= 1e-10


@pytest.mark.timeout(400)
def test_c4_batch_instances_match_oracle(slhjb):
    """The uneven 64-instance two-asset batch (65^2 ... 513^2, 50 implicit steps) in one hjb_solve_batch; four of
    its 65^2 instances against the oracle: values to the parity bound and policies at every clear decision."""
    insts = workloads.config_c4()
    log(f"C4 batch: {len(insts)} instances, {sum(i.N for i in insts)} nodes")
    Ub, pb, st = _run_batch(slhjb, insts, slhjb.Options(precision=1))
    small = [b for b, inst in enumerate(insts) if inst.n[0] == 65][:4]
    for b in small:
        inst = insts[b]
        ref = oracle.march(inst, keep_policies=True, keep_values=True)
        rel = np.max(np.abs(Ub[b] - ref["U"])) / np.max(np.abs(ref["U"]))
        log(f"  instance {b} ({inst.n[0]}^2): batch pi={st[b].pi_total} krylov={st[b].krylov_total} rel {rel:.2e}")
        assert st[b].steps_done == len(inst.dts)
        assert rel <= 1e-10
        check_march_policies(inst, ref, pb[b], log=log)


def _run_batch_tuned(slhjb, insts, opts, widths=None, cache=None):
    bt = slhjb.Batch(insts, opts)
    chosen = None
    if widths is not None:
        bt.set_tile_widths(widths)
    if cache is not None:
        chosen = bt.autotune(cache)
    g, psi, f0, f1 = (to_dev(bt.concat(k)) for k in ("g", "psi", "f0", "f1"))
    U = torch.empty_like(g)
    pol = torch.empty((len(insts[0].dts), bt.total), dtype=torch.int16, device="cuda")
    st = bt.solve(g, psi, f0, f1, insts[0].dts, insts[0].thetas, 1.0, U, pol)
    out = [to_np(u) for u in bt.split(U)]
    pols = [to_np(pol[:, o:o + inst.N]) for inst, o in zip(insts, bt.offsets)]
    bt.close()
    return out, pols, st, chosen


def test_batch_per_instance_tile_widths(slhjb):
    """Each instance of a batch on its own tile shape: the launch lists follow the instances' tiles, and the
    results meet the oracle and the uniform-width batch (partial sums follow the tiles, so agreement is to the
    certificate, not bitwise)."""
    insts = _batch_2d()
    widths = [16, 64, 128, 32, 16, 64]
    opts = slhjb.Options(precision=1, max_levels=0)
    Uw, pw, st, _ = _run_batch_tuned(slhjb, insts, opts, widths=widths)
    Uu, pu, _ = _run_batch(slhjb, insts, opts)
    for b, inst in enumerate(insts):
        ref = oracle.march(inst, keep_policies=True, keep_values=True)
        rel = np.max(np.abs(Uw[b] - ref["U"])) / np.max(np.abs(ref["U"]))
        relu = np.max(np.abs(Uw[b] - Uu[b])) / np.max(np.abs(Uu[b]))
        check_march_policies(inst, ref, pw[b], log=log)
        log(f"  {inst.name} width {widths[b]}: pi={st[b].pi_total} krylov={st[b].krylov_total} rel vs oracle "
            f"{rel:.2e}, vs uniform {relu:.2e}")
        assert rel <= 1e-10 and relu <= 1e-10
    with pytest.raises(slhjb.HJBError):
        bt = slhjb.Batch(insts, opts)
        try:
            bt.set_tile_widths([16, 64, 128, 32, 16, 48])
        finally:
            bt.close()


def test_batch_autotune(slhjb, tmp_path):
    """The autotuner over a batch: one timing run per distinct instance key, widths from the cache on the
    second call, and a solve on the chosen shapes that meets the oracle."""
    insts = _batch_2d()[:4]
    cache = str(tmp_path / "tune.jsonl")
    opts = slhjb.Options(precision=1)
    U1, p1, st, w1 = _run_batch_tuned(slhjb, insts, opts, cache=cache)
    _, _, _, w2 = _run_batch_tuned(slhjb, insts, opts, cache=cache)
    log(f"  autotuned widths {w1}, from the cache {w2}")
    assert all(w in (16, 32, 64, 128) for w in w1)
    assert w1 == w2
    lines = open(cache).read().splitlines()
    assert 1 <= len(lines) <= len(insts)
    for b, inst in enumerate(insts):
        ref = oracle.march(inst, keep_policies=True, keep_values=True)
        rel = np.max(np.abs(U1[b] - ref["U"])) / np.max(np.abs(ref["U"]))
        check_march_policies(inst, ref, p1[b], log=log)
        assert rel <= 1e-10
