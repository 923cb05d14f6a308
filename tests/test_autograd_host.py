"""Host logic of the differentiable wrappers (paper_2509_22975_amd.autograd),
on the CPU with the library calls replaced by stand-ins: a solve that stopped
at its iteration cap makes the forward (ground state) or the backward
(response solve) raise instead of returning a value or gradient of an
unconverged state."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")


class _Info:
    def __init__(self, converged):
        self.converged = converged
        self.iters = 7
        self.residual = 1e-3


class _Op:
    def __init__(self, *a, **k):
        pass

    def contract(self, psi):
        return np.zeros(3), np.zeros(2), np.zeros(2)

    def close(self):
        pass


def _model():
    return W.Model(2, [(0, 1, -1.0)], np.array([4.0, 4.0]), np.array([-2.0, -2.0]), 1, 1, "two")


def test_ground_energy_refuses_an_unconverged_ground_state(monkeypatch):
    from paper_2509_22975_amd import autograd as ag
    monkeypatch.setattr(ag, "Operator", _Op)
    monkeypatch.setattr(ag, "lanczos_ground",
                        lambda op, **kw: (-1.0, torch.zeros(4, dtype=torch.float64), None, None,
                                          _Info(False)))
    t = torch.tensor([-1.0], dtype=torch.float64, requires_grad=True)
    U = torch.tensor([4.0, 4.0], dtype=torch.float64)
    eps = torch.tensor([-2.0, -2.0], dtype=torch.float64)
    with pytest.raises(ag.NotConvergedError):
        ag.ground_energy(_model(), None, t, U, eps)
    # a converged solve goes through
    monkeypatch.setattr(ag, "lanczos_ground",
                        lambda op, **kw: (-1.0, torch.zeros(4, dtype=torch.float64), None, None,
                                          _Info(True)))
    e = ag.ground_energy(_model(), None, t, U, eps)
    assert float(e) == -1.0


def test_green_backward_refuses_an_unconverged_response(monkeypatch):
    from paper_2509_22975_amd import autograd as ag
    monkeypatch.setattr(ag, "Operator", _Op)
    monkeypatch.setattr(ag, "lanczos_ground",
                        lambda op, **kw: (-1.0, torch.zeros(4, dtype=torch.float64), None, None,
                                          _Info(True)))

    class _Keep:
        def close(self):
            pass

    monkeypatch.setattr(ag, "band_lanczos_green",
                        lambda *a, **k: (np.zeros((2, 1, 1), complex), _Info(True), _Keep()))
    monkeypatch.setattr(ag, "band_green_vjp",
                        lambda *a, **k: (np.zeros(1), np.zeros(2), np.zeros(2), _Info(False)))
    t = torch.tensor([-1.0], dtype=torch.float64, requires_grad=True)
    U = torch.tensor([4.0, 4.0], dtype=torch.float64)
    eps = torch.tensor([-2.0, -2.0], dtype=torch.float64)
    e0, G = ag.green_function(_model(), None, t, U, eps, [0], [0], [1.0, 3.0])
    loss = G.abs().sum() + e0
    with pytest.raises(ag.NotConvergedError):
        loss.backward()
