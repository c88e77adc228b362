"""Least-squares refinement logic on the CPU with a dense operator.

``refine_with`` is operator-generic; with a small random complex matrix A as
the echo model (float64 on the CPU) its conjugate-gradient form must reach the
least-squares solution of numpy's lstsq within n steps (CGNR terminates in at
most n steps in exact arithmetic), steepest descent must decrease the residual
monotonically, and a run interrupted after a few steps and resumed from its
checkpoint must end bit for bit where the uninterrupted run ends.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2109_02842_amd import autograd as ag  # noqa: E402


def _problem(seed=3, m=40, n=8):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) / np.sqrt(2)
    x_true = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    s = A @ x_true + 0.05 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    At = torch.from_numpy(A)
    ops = (lambda x: At @ x, lambda r: At.conj().T @ r, lambda x: At @ x)
    return A, torch.from_numpy(s), ops


def test_cgnr_reaches_the_least_squares_solution():
    A, s, (adj, fwd, model) = _problem()
    x, hist = ag.refine_with(adj, fwd, s, (A.shape[1],), steps=A.shape[1] + 2, method="cg")
    ref = np.linalg.lstsq(A, s.numpy(), rcond=None)[0]
    assert np.linalg.norm(x.numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    assert abs(hist[-1] - np.linalg.norm(A @ ref - s.numpy())) <= 1e-9 * hist[-1]


def test_steepest_descent_decreases_the_residual():
    A, s, (adj, fwd, model) = _problem(seed=4)
    x, hist = ag.refine_with(adj, fwd, s, (A.shape[1],), steps=25, method="sd", model=model)
    assert len(hist) == 26
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    ref = np.linalg.lstsq(A, s.numpy(), rcond=None)[0]
    assert hist[-1] <= 1.05 * np.linalg.norm(A @ ref - s.numpy())


@pytest.mark.parametrize("method", ["cg", "sd"])
def test_resume_from_checkpoint_matches_an_uninterrupted_run(method, tmp_path):
    A, s, (adj, fwd, model) = _problem(seed=5)
    shape = (A.shape[1],)
    x_ref, h_ref = ag.refine_with(adj, fwd, s, shape, steps=7, method=method, model=model)
    ck = str(tmp_path / "refine.pt")
    ag.refine_with(adj, fwd, s, shape, steps=3, method=method, model=model, checkpoint=ck)
    x, h = ag.refine_with(adj, fwd, s, shape, steps=7, method=method, model=model, checkpoint=ck, resume=True)
    assert torch.equal(x, x_ref)
    assert h == h_ref
    state = torch.load(ck, weights_only=True)
    assert state["step"] == 7 and state["method"] == method
    with pytest.raises(ValueError):
        ag.refine_with(adj, fwd, s, shape, steps=9, method="sd" if method == "cg" else "cg", model=model,
                       checkpoint=ck, resume=True)
