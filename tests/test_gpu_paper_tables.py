"""The paper's Problems A and B (Section 2.4) on the GPU path: per-node sigma (Problem A), per-control
sources (Problem B), explicit (theta = 0) and implicit (theta = 1) steps.

On small grids the GPU marches equal the oracle's (explicit: bit for bit, one search and one update
per step; implicit: to the 1e-10 parity bound).  On larger grids the GPU's L-infinity errors at t = T
over the whole grid are compared with the values the paper prints (tests/golden/paper_tables.json):
Tab:Linf_matrix_40 / Tab:Linf_exp_trunc_40_B (explicit, truncation) and Tab:Linf_imp_trunc_40
(implicit, truncation, dt = T), to the three digits printed, and the explicit scheme with dt = dx/4
blows up at N_x = 321 as printed (Cor. cor:CFL).  The shifted box of Remark rem:two-over (time-dependent
boundary data, two-sided overstepping) reproduces Table Tab:shifted, blow-ups included.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import log, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
DTS = {"dt=T": lambda h: 0.5, "dt=dx/4": lambda h: h / 4, "dt=dx^1.5": lambda h: h ** 1.5, "dt=dx^2": lambda h: h * h}


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _make(prob, Nx, col, theta):
    h = 2 * math.pi / (Nx - 1)
    if prob == "A-shifted":
        return workloads.problem_a(Nx, dt=DTS[col](h), theta=theta, lo_shift=7 * math.pi / 8)
    mk = workloads.problem_a if prob == "A" else workloads.problem_b
    return mk(Nx, dt=DTS[col](h), theta=theta)


def _gpu_march(slhjb, inst, precision=0):
    solver = slhjb.Solver.from_instance(inst, slhjb.Options(precision=precision))
    g = to_dev(inst.g)
    U = torch.empty_like(g)
    psi1 = None if inst.psi1 is None else to_dev(inst.psi1)
    st = solver.solve(g, to_dev(inst.psi), to_dev(np.ascontiguousarray(inst.f0)), to_dev(np.ascontiguousarray(inst.f1)),
                      inst.dts, inst.thetas, inst.s, U, psi1=psi1)
    solver.close()
    return to_np(U), st


def _err(inst, U):
    return float(np.max(np.abs(U - inst.exact(inst.T, inst.coords()))))


@pytest.mark.parametrize("prob", ["A", "B", "A-shifted"])
@pytest.mark.parametrize("Nx,col", [(41, "dt=dx^2"), (41, "dt=T"), (81, "dt=dx^1.5")])
def test_explicit_march_bit_exact(slhjb, prob, Nx, col):
    inst = _make(prob, Nx, col, 0.0)
    log(f"explicit problem {prob} N_x={Nx} {col}: {len(inst.dts)} steps")
    ref = oracle.march(inst)["U"]
    U, st = _gpu_march(slhjb, inst)
    np.testing.assert_array_equal(U, ref)


@pytest.mark.parametrize("prob", ["A", "B"])
@pytest.mark.parametrize("Nx", [41, 81])
@pytest.mark.parametrize("precision", [0, 1])
def test_implicit_march_matches_oracle(slhjb, prob, Nx, precision):
    inst = _make(prob, Nx, "dt=T", 1.0)
    ref = oracle.march(inst)["U"]
    U, st = _gpu_march(slhjb, inst, precision)
    rel = float(np.max(np.abs(U - ref)) / np.max(np.abs(ref)))
    log(f"implicit problem {prob} N_x={Nx} precision={precision}: pi={st.pi_total} krylov={st.krylov_total} rel={rel:.2e}")
    assert rel <= 1e-10


EXPLICIT_CASES = [("A", "dt=T", 161), ("A", "dt=T", 321), ("A", "dt=T", 641), ("A", "dt=dx^2", 161),
                  ("A", "dt=dx^2", 321), ("A", "dt=dx^1.5", 321), ("A", "dt=dx^1.5", 641),
                  ("B", "dt=T", 321), ("B", "dt=T", 641), ("B", "dt=dx^2", 161), ("B", "dt=dx^2", 321),
                  ("B", "dt=dx^1.5", 641)]


@pytest.mark.parametrize("prob,col,Nx", EXPLICIT_CASES, ids=[f"{p}-{c}-{n}" for p, c, n in EXPLICIT_CASES])
def test_explicit_table_values(slhjb, prob, col, Nx):
    inst = _make(prob, Nx, col, 0.0)
    U, st = _gpu_march(slhjb, inst)
    e = _err(inst, U)
    ref = GOLDEN[f"explicit_truncation_{prob}"][col][str(Nx)]
    log(f"explicit problem {prob} {col} N_x={Nx}: {len(inst.dts)} steps, error {e:.3e} (paper {ref:.2e})")
    assert e == pytest.approx(ref, rel=6e-3)


@pytest.mark.parametrize("prob", ["A", "B"])
def test_explicit_cfl_blowup(slhjb, prob):
    """dt = dx/4 with truncation violates the CFL condition of Cor. cor:CFL at N_x = 321: the paper prints
    errors of 1e+23 (A) and 1e+43 (B)."""
    inst = _make(prob, 321, "dt=dx/4", 0.0)
    U, st = _gpu_march(slhjb, inst)
    e = _err(inst, U)
    log(f"explicit problem {prob} dt=dx/4 N_x=321: error {e:.3e}")
    assert not np.isfinite(e) or e > 1e10


@pytest.mark.parametrize("Nx", [161, 321, 641])
def test_implicit_table_values_problem_a(slhjb, Nx):
    inst = _make("A", Nx, "dt=T", 1.0)
    U, st = _gpu_march(slhjb, inst, precision=1)
    e = _err(inst, U)
    ref = GOLDEN["implicit_truncation_A"]["dt=T"][str(Nx)]
    log(f"implicit problem A N_x={Nx}: pi={st.pi_total} krylov={st.krylov_total} error {e:.3e} (paper {ref:.2e})")
    assert e == pytest.approx(ref, rel=5e-3)


@pytest.mark.parametrize("Nx", [161, 321, 641])
def test_implicit_problem_b_report(slhjb, Nx):
    """Problem B, implicit, dt = T: reported beside the printed values (parity unpinned above N_x = 81,
    where the oracle itself differs from the print by a few percent); the error must still decrease."""
    inst = _make("B", Nx, "dt=T", 1.0)
    U, st = _gpu_march(slhjb, inst, precision=1)
    e = _err(inst, U)
    ref = GOLDEN["implicit_truncation_B"]["dt=T"][str(Nx)]
    log(f"implicit problem B N_x={Nx}: error {e:.3e} (paper {ref:.2e}, ratio {e / ref:.3f})")
    assert 0.5 * ref < e < 2.0 * ref


def _shifted_err(inst, U):
    X = inst.coords()
    e = np.abs(U - inst.exact(inst.T, X))
    lo, hi = 3 * math.pi / 8 - 1e-12, 11 * math.pi / 8 + 1e-12
    m = (X[0] >= lo) & (X[0] <= hi) & (X[1] >= lo) & (X[1] <= hi)
    return float(np.max(e)), float(np.max(e[m]))


SHIFTED_CASES = [("dt=T", 161), ("dt=T", 321), ("dt=T", 641), ("dt=dx^2", 161), ("dt=dx^2", 321),
                 ("dt=dx/4", 161), ("dt=dx^1.5", 161)]


@pytest.mark.parametrize("col,Nx", SHIFTED_CASES, ids=[f"{c}-{n}" for c, n in SHIFTED_CASES])
def test_shifted_domain_table_values(slhjb, col, Nx):
    """Table Tab:shifted (Remark rem:two-over): Problem A on [-pi/8, 15pi/8]^2 with the time-dependent boundary
    data psi(t) = (3/2 - t) sin x1 sin x2, explicit scheme with truncation.  Both sides of the diffusion stencil
    overstep near the corner (-pi/8, -pi/8), so dt = dx/4 and dt = dx^(3/2) blow up (Cor. cor:CFL) while dt = dx^2
    converges; whole-grid and interior errors to the three printed digits."""
    inst = _make("A-shifted", Nx, col, 0.0)
    U, st = _gpu_march(slhjb, inst)
    whole, inner = _shifted_err(inst, U)
    gw = GOLDEN["explicit_truncation_A_shifted"]["whole grid"][col][str(Nx)]
    gi = GOLDEN["explicit_truncation_A_shifted"]["[3pi/8, 11pi/8]^2"][col][str(Nx)]
    log(f"shifted problem A {col} N_x={Nx}: {len(inst.dts)} steps, errors {whole:.3e} / {inner:.3e} "
        f"(paper {gw:.2e} / {gi:.2e})")
    assert whole == pytest.approx(gw, rel=6e-3)
    assert inner == pytest.approx(gi, rel=6e-3)


def test_shifted_domain_blowup_at_321(slhjb):
    """dt = dx/4 at N_x = 321 on the shifted box: the paper prints 6.73e+103 (whole grid) and 7.99e+47 (interior)."""
    inst = _make("A-shifted", 321, "dt=dx/4", 0.0)
    U, st = _gpu_march(slhjb, inst)
    whole, inner = _shifted_err(inst, U)
    log(f"shifted problem A dt=dx/4 N_x=321: errors {whole:.3e} / {inner:.3e}")
    assert not np.isfinite(whole) or whole > 1e90
    assert not np.isfinite(inner) or inner > 1e40
