"""Pins of the differentiable FP64 reference (oracle/torch_ref.py) used to
check the GPU adjoint: its forward equals the C oracle's step by step, and
its autograd gradient equals central differences of the C oracle (a second,
independent implementation) for the relaxation time, gravity and initial
particle velocities, with soft contacts engaged and particles near walls."""
import numpy as np
import pytest
import torch

from oracle import torch_ref as TR


def _case(lattice, seed):
    rng = np.random.default_rng(seed)
    if lattice == 9:
        n = (24, 20, 1)
        X = np.array([[6.0, 6.42, 12.0, 12.3, 18.0, 3.0, 20.0, 9.0],
                      [8.0, 8.1, 12.0, 12.38, 6.0, 0.2, 15.0, 17.0]])
    else:
        n = (12, 10, 9)
        X = np.array([[4.0, 4.45, 8.0, 6.0, 2.0],
                      [4.0, 4.05, 6.0, 7.0, 5.0],
                      [4.0, 4.1, 5.0, 0.22, 7.0]])
    D = X.shape[0]
    X = X + 0.01 * rng.standard_normal(X.shape)
    npart = X.shape[1]
    d = np.full(npart, 0.5)
    rp = rng.uniform(1.8, 3.0, npart)
    U = 1e-3 * rng.standard_normal((D, npart))
    return n, X, U, d, rp


def _oracle_rollout(orc, lattice, n, tau, g, X, U, d, rp, steps, n_sub):
    D = 2 if lattice == 9 else 3
    grav = [0.0, 0.0, 0.0]
    grav[D - 1] = -g
    oc = orc.make_cfg(lattice=lattice, n=n, tau=tau, gravity=grav, contact="soft", k_soft=2e-3,
                      skin=0.05, n_sub=n_sub, two_way=1, bin_log2=0)
    f = orc.rest_state(oc)
    for _ in range(steps):
        r = orc.step(oc, f, X, U, d, rp)
        f, X, U = r["f"], r["X"], r["U"]
        assert r["nskin"] == 0
    return f, X, U


@pytest.mark.parametrize("lattice,n_sub", [(9, 1), (9, 3), (19, 4), (15, 2)])
def test_forward_matches_c_oracle(orc, lattice, n_sub):
    n, X, U, d, rp = _case(lattice, 3)
    tau, g, steps = 0.7, 1e-3, 12
    f_o, X_o, U_o = _oracle_rollout(orc, lattice, n, tau, g, X, U, d, rp, steps, n_sub)
    ref = TR.Ref(lattice, n, d, rp, k_soft=2e-3, contact="soft", n_sub=n_sub)
    D = ref.D
    gvec = torch.zeros(D, dtype=torch.float64)
    gvec[D - 1] = -g
    f, Xr, Ur = ref.rollout(torch.tensor(X), torch.tensor(U), tau, gvec, steps)
    assert np.abs(f.numpy().reshape(-1) - f_o).max() <= 1e-14
    assert np.abs(Xr.numpy() - X_o).max() <= 1e-12
    assert np.abs(Ur.numpy() - U_o).max() <= 1e-14
    # the case really exercises the contacts
    Fc = ref.contact_force(torch.tensor(X))
    assert (Fc.abs().sum(0) > 0).sum() >= 3


def test_gradient_matches_c_oracle_central_differences(orc):
    lattice = 9
    n, X, U, d, rp = _case(lattice, 5)
    tau, g, steps = 0.7, 1e-3, 15
    ref = TR.Ref(lattice, n, d, rp, k_soft=2e-3, contact="soft", n_sub=1)
    t_tau = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    t_g = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    t_U = torch.tensor(U, requires_grad=True)
    X0 = torch.tensor(X)
    gvec = torch.stack([torch.zeros((), dtype=torch.float64), -t_g])
    _, XT, _ = ref.rollout(X0, t_U, t_tau, gvec, steps)
    J = (XT[1] - X0[1]).mean()
    J.backward()

    def J_oracle(tau_, g_, U_):
        _, XT_, _ = _oracle_rollout(orc, lattice, n, tau_, g_, X, U_, d, rp, steps, 1)
        return (XT_[1] - X[1]).mean()

    def central(fp, fm, h):
        return (fp - fm) / (2 * h)

    h = 1e-4
    fd_tau = central(J_oracle(tau + h, g, U), J_oracle(tau - h, g, U), h)
    h = 1e-6
    fd_g = central(J_oracle(tau, g + h, U), J_oracle(tau, g - h, U), h)
    assert abs(t_tau.grad.item() - fd_tau) <= 1e-6 * abs(fd_tau) + 1e-12
    assert abs(t_g.grad.item() - fd_g) <= 1e-6 * abs(fd_g)
    h = 1e-6
    for (a, p) in ((0, 0), (1, 0), (1, 1), (0, 3), (1, 5)):
        Up, Um = U.copy(), U.copy()
        Up[a, p] += h
        Um[a, p] -= h
        fd = central(J_oracle(tau, g, Up), J_oracle(tau, g, Um), h)
        ad = t_U.grad[a, p].item()
        assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-12, (a, p, ad, fd)
