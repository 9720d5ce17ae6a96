"""Wiener filter under the error bound of Sect. 2.2 (mfwf_solve_bounded).

The lambda sequence depends on the data, so parity replays it: the run reports the lambda of
every iteration and the oracle iterates with the same sequence.  The bound itself,
chi^2(lambda, x) <= b after every iteration, is checked on the reported trace, and the end
result against the dense fixed point of the iteration.  T, Q, U plans replay against
oracle.solve_pol.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import dense
from paper_1210_4931_amd import workloads as W
from tests.gpu_util import dev, rel, rel_alm, temperature_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_4931_amd import mfwf
    mfwf.load()
    return mfwf


def _plan(mf, nside, lmax, seed=0, dtype="f64", max_batch=1):
    wl, d, M = temperature_problem(nside, lmax, seed)
    plan = mf.Plan(nside, lmax, max_batch=max_batch, dtype=dtype)
    plan.set_covariances(wl.cl, dev(1.0 / wl.noise_var), dev(wl.mask, torch.uint8))
    return plan, wl, d, M


def test_bounded_replay_and_bound(mf):
    nside, lmax = 32, 64
    plan, wl, d, M = _plan(mf, nside, lmax)
    s_alm, s_map, info, trace, nup, reached = plan.solve_bounded(dev(d[None]), max_iters=600)
    lam, E, b = trace[:, 0], trace[:, 1], trace[:, 2]
    print("iterations", len(lam), "b updates", nup, "reached 1", reached, "lambda", lam[:5],
          "...", lam[-3:], "chi2/ndof", info[0].chi2 / info[0].n_dof)
    up = np.nonzero(np.diff(lam) > 0.0)[0]
    print("lambda rises after iterations", up, "lam", lam[up], "->", lam[up + 1],
          "E/b there", (E / b)[up], "b updates at", np.nonzero(np.diff(b) != 0)[0])
    print("max E/b", np.max(E / b), "at", np.argmax(E / b))
    assert lam[0] > 1.0
    # the bound after every iteration, up to the quadrature gap of the pixelised sphere (an
    # iteration at fixed lambda lowers chi^2(lambda, x) only up to that gap); lambda rises
    # only right after an iteration that exceeded b, to restore the bound
    assert np.all(E <= b * (1.0 + 1e-4)), np.max(E / b)
    assert np.all(E[up] > b[up])
    ref_alm, ref_map, dg = oracle.solve(nside, lmax, wl.cl, M, M * d, lam=lam, diag=True)
    assert rel_alm(s_alm.cpu().numpy()[0], ref_alm, lmax) < 1e-10
    assert rel(s_map.cpu().numpy()[0], ref_map) < 1e-10
    # the oracle's chi^2(lambda_k, x_k) along the replay is the trace's, excursions included
    assert rel(dg[:, 0], E) < 1e-9


def test_bounded_f32_batch_replay(mf):
    nside, lmax = 32, 64
    plan, wl, d, M = _plan(mf, nside, lmax, seed=1, dtype="f32", max_batch=2)
    rng = np.random.default_rng(3)
    ds = np.stack([d, d + rng.standard_normal(d.size) * np.sqrt(wl.noise_var)])
    s_alm, s_map, info, trace, nup, reached = plan.solve_bounded(dev(ds), max_iters=250)
    for b in range(2):
        ref_alm, ref_map = oracle.solve(nside, lmax, wl.cl, M, M * ds[b], lam=trace[:, 0])
        assert rel_alm(s_alm.cpu().numpy()[b], ref_alm, lmax) < 1e-5
        assert rel(s_map.cpu().numpy()[b], ref_map) < 1e-5


def test_bounded_solve_reaches_one_near_the_fixed_point(mf):
    nside, lmax = 16, 32
    plan, wl, d, M = _plan(mf, nside, lmax, seed=2)
    s_alm, _, info, trace, nup, reached = plan.solve_bounded(dev(d[None]), max_iters=4000)
    assert reached and trace[-1, 0] == 1.0
    n = len(trace)
    fp = dense.Problem(nside, lmax, wl.cl, M).messenger_fixed_point(M * d)
    err = rel(dense.alm_to_real(s_alm.cpu().numpy()[0], lmax), fp)
    s_plain, _, _ = plan.solve(dev(d[None]), iters=n)
    err_plain = rel(dense.alm_to_real(s_plain.cpu().numpy()[0], lmax), fp)
    print("iterations", n, "b updates", nup, "error vs fixed point", err, "plain", err_plain)
    assert err < err_plain


def _pol_problem(mf, nside, lmax, seed, dtype, max_batch):
    w = W.config3(seed, nside, lmax, ndisc=10, band_z=0.15, nu=10)
    d = w.data_from_signal_maps(oracle.alm2map_pol(nside, lmax, w.signal_alm))
    plan = mf.Plan(nside, lmax, max_batch=max_batch, spin=2, dtype=dtype)
    plan.set_covariances(w.cl4, dev(w.ninv6), dev(w.mask, torch.uint8))
    M6 = w.M6()
    Mb = M6[:, [0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(-1, 3, 3)
    return plan, w, d, M6, Mb


def _rel_teb(a, ref, lmax):
    _, ms = W.alm_l_m(lmax)
    w = np.sqrt(np.where(ms == 0, 1.0, 2.0))
    return rel(a * w, ref * w)


def _pix_term(Mb, rho, s_map, tau, lam):
    """sum over observed blocks of q^T [M + (lam - 1) tau M^2]^-1 q, q = rho - M s."""
    obs = np.linalg.det(Mb) > 0
    M = Mb[obs]
    q = rho.T[obs] - np.einsum("pij,pj->pi", M, s_map.T[obs])
    B = M + (lam - 1.0) * tau * (M @ M)
    return float(np.sum(q * np.linalg.solve(B, q[..., None])[..., 0]))


def test_bounded_pol_replay_bound_and_b_update(mf):
    """T, Q, U (spin 2), FP64: the bound on the trace, the oracle's replay, and every raise of
    b against chi^2 - (lambda - 1) dP/dlambda with the derivative of the pixel term taken by
    finite differences on the replayed iterate.

    The bound's margin is wider than for temperature: with correlated 3x3 noise blocks an
    iteration at fixed lambda can raise chi^2(lambda, x) after lambda has dropped, because the
    analysis Omega Y^T inverts the synthesis only up to the pixelisation.  The oracle shows the
    same rise (over ten iterations at lambda 3 after eighty at lambda 10: 1.3e-3 at nside 16,
    8.8e-4 at nside 32, none at nside 64, lmax = 2 nside), and the trace's chi^2 equals the
    oracle's replay to 1e-9, excursions included."""
    nside, lmax = 32, 64
    plan, w, d, M6, Mb = _pol_problem(mf, nside, lmax, 0, "f64", 1)
    s_alm, s_map, info, trace, nup, reached = plan.solve_bounded(dev(d[None]), max_iters=800)
    lam, E, b = trace[:, 0], trace[:, 1], trace[:, 2]
    ups = np.nonzero(np.diff(b) != 0)[0]
    print("iterations", len(lam), "b updates", nup, "at", ups, "reached 1", reached,
          "lambda", lam[:4], "...", lam[-3:], "chi2/ndof", info[0].chi2 / info[0].n_dof)
    assert lam[0] > 1.0 and info[0].n_dof == 3 * int(w.mask.sum())
    up = np.nonzero(np.diff(lam) > 0.0)[0]
    assert np.all(E <= b * (1.0 + 2e-3)), np.max(E / b)
    assert np.all(E[up] > b[up])
    rho = np.einsum("pij,jp->ip", Mb, d)
    ref_alm, ref_map, dg = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=lam, diag=True)
    assert _rel_teb(s_alm.cpu().numpy()[0], ref_alm, lmax) < 1e-10
    assert rel(s_map.cpu().numpy()[0], ref_map) < 1e-10
    assert rel(dg[:, 0], E) < 1e-9
    assert len(ups) == nup
    tau = info[0].tau
    for u in ups[:4]:
        _, x_u = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=lam[:u + 1])
        # five-point central difference, error O(h^4)
        h = 1e-3 * (lam[u] - 1.0)
        P = [_pix_term(Mb, rho, x_u, tau, lam[u] + k * h) for k in (-2, -1, 1, 2)]
        dP = (P[0] - 8.0 * P[1] + 8.0 * P[2] - P[3]) / (12.0 * h)
        want = E[u] - (lam[u] - 1.0) * dP
        assert b[u + 1] == pytest.approx(want, rel=1e-9), (u, b[u + 1], want)


def test_bounded_pol_f32_batch_replay(mf):
    nside, lmax = 16, 32
    plan, w, d, M6, Mb = _pol_problem(mf, nside, lmax, 1, "f32", 2)
    rng = np.random.default_rng(4)
    ds = np.stack([d, d + rng.standard_normal(d.shape)])
    s_alm, s_map, info, trace, nup, reached = plan.solve_bounded(dev(ds), max_iters=250)
    for k in range(2):
        rho = np.einsum("pij,jp->ip", Mb, ds[k])
        ref_alm, ref_map = oracle.solve_pol(nside, lmax, w.cl4, M6, rho, lam=trace[:, 0])
        assert _rel_teb(s_alm.cpu().numpy()[k], ref_alm, lmax) < 1e-5
        assert rel(s_map.cpu().numpy()[k], ref_map) < 1e-5


def test_bounded_errors(mf):
    from paper_1210_4931_amd.mfwf import MFWFError
    plan, wl, d, M = _plan(mf, 8, 16)
    with pytest.raises(MFWFError):
        plan.solve_bounded(dev(d[None]), m_sigma=-1.0)
    with pytest.raises(MFWFError, match="status -4"):
        mf.Plan(4, 8, spin=2).solve_bounded(torch.zeros((1, 3, 192), dtype=torch.float64,
                                                        device="cuda"))
