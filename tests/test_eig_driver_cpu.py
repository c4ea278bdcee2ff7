"""CPU checks of the host driver's algebra (moment recurrence of Algorithm 1, restarts,
reduced pencil) against the oracle's step-by-step Algorithm 1, using a stand-in mesh whose
sweeps are dense products with the oracle's operator (no GPU involved)."""
import numpy as np
import pytest
import torch

import synth
from oracle import method as M
from paper_1906_03938_amd.eig import ContourSolver


class DenseMesh:
    """Sweeps computed from dense oracle matrices; inputs and outputs are CPU tensors."""

    def __init__(self, op):
        self.op = op
        self.n = op.n

    def contour_moments(self, z, W, V):
        V = V.numpy()
        out = sum(np.asarray(W)[j][:, None, None] * self.op.dense(z[j]) @ V for j in range(len(z)))
        return torch.from_numpy(np.ascontiguousarray(out.reshape(np.asarray(W).shape[1], self.n, -1)))

    def rr_project(self, z, U):
        U = U.numpy()
        return torch.from_numpy(np.stack([U.conj().T @ self.op.dense(zj) @ U for zj in z]))

    def assemble_apply(self, kappas, V):
        V = V.numpy()
        return torch.from_numpy(np.stack([self.op.dense(k) @ V for k in kappas]))


class CpuSolver(ContourSolver):
    def _dev(self, a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))


@pytest.fixture(scope="module")
def setup():
    xyz, tri = synth.icosphere(1)
    op = M.Operator(xyz, tri)
    return op, DenseMesh(op)


def _unit_cols(u):
    return u / np.linalg.norm(u, axis=0, keepdims=True)


def _oracle_iterate(op, c, R, N, v, u, q):
    s, w = M.circle_nodes(c, R, N)
    Bs = [w[j] * op.dense(s[j]) for j in range(N)]
    for _ in range(q):
        v, u = M.inverse_power_step(Bs, s, c, v, u)
        sc = 1.0 / np.linalg.norm(u, axis=0)
        u = u * sc
        v = [vi * sc for vi in v]
    return u


def test_moment_recurrence_equals_algorithm1(setup):
    op, mesh = setup
    c, R, N, q = 4.0, 1.5, 32, 6
    u0 = synth.probe_block(op.n, 5, seed=3)
    solver = CpuSolver(mesh, c, R, N, q=q)
    u = solver.inverse_iteration(u0)
    s, _ = M.circle_nodes(c, R, N)
    uo = _oracle_iterate(op, c, R, N, [u0 / (c - s[i]) for i in range(N)], u0, q)
    assert np.abs(_unit_cols(u) - uo).max() < 1e-12


def test_restart_recurrence_equals_algorithm1(setup):
    op, mesh = setup
    c, R, N, q = 4.0, 1.5, 32, 5
    x = synth.probe_block(op.n, 3, seed=4)
    lam = np.array([3.3 + 0.01j, 4.7, 4.1 - 0.2j])
    solver = CpuSolver(mesh, c, R, N, q=q)
    u = solver.inverse_iteration(x, lam)
    s, _ = M.circle_nodes(c, R, N)
    uo = _oracle_iterate(op, c, R, N, [x / (lam[None, :] - s[i]) for i in range(N)], x, q)
    assert np.abs(_unit_cols(u) - uo).max() < 1e-12


def test_driver_eigenvalues_match_oracle(setup):
    op, mesh = setup
    V = synth.probe_block(op.n, 8, seed=1)
    lam, X, res, outer = CpuSolver(mesh, 4.0, 1.5, 32, q=10, tol=1e-12).solve(V)
    lo, _, reso, _, _ = M.subspace_iteration(op, 4.0, 1.5, 32, V, q=10, tol=1e-12)
    assert res.max() <= 1e-12 and lam.size == lo.size == 4
    assert np.abs(np.sort_complex(lam) - np.sort_complex(lo)).max() <= 1e-10 * np.abs(lo).max()
