"""GPU low modes of D^+D and coarse-space coverage against the oracle (paper
Sec. 2, Fig. 1 right).

* Lanczos on (D^+D)^-1 through (squared-operator) multigrid solves gives the lowest eigenvalues
  of the oracle's dense D^+D to 1e-9, eigenvectors that match the oracle's
  ones up to a phase, and reported residuals below 1e-6;
* the coverage |P R e|^2 / |e|^2 of the oracle's eigenvectors by the GPU's
  basis equals the oracle's coverage with that basis to 1e-12;
* a basis made of the lowest four modes (cut into blocks) covers each of them
  entirely, on the GPU as in the oracle.
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion, prepare_gauge, random_starts
from oracle import dwf
from oracle import lowmodes as olm
from oracle import transfer as ot

pytestmark = pytest.mark.gpu

L, LS, MF, M5, BLOCK = (2, 2, 2, 4), 4, 0.05, 1.8, (2, 2, 2, 2)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def dense():
    U = prepare_gauge(L, 0.4, 80)
    A = dwf.DWF(U, M5, MF)
    shape = tuple(L[::-1]) + (LS, 4, 3)
    lam, E = olm.lowest_modes(A, shape, 16)
    return U, lam, E


@pytest.mark.parametrize("squared", [True])
def test_lanczos_low_modes_match_dense_eigh(cuda, dense, squared):
    """The Lanczos solves run on the squared-operator multigrid: on this 2^3 x 4
    lattice the 9-point one stalls near |r|/|b| ~ 1 on some Lanczos
    right-hand sides (restarted flexible GCR; its plain solves converge)."""
    import paper_1205_2933_amd as mg
    U, lam, E = dense
    nvec, nev = 16, 6  # with 8 the restarted solves stall on this lattice (the oracle's too)
    h = mg.Handle(L, LS, M5, MF)
    mg.mgdwf_set_gauge(h, dev(U))
    prm = mg.make_mg_params(BLOCK, nvec, sweeps=1, sweep0_iters=60, nu_pre=4, nu_post=4, coarse_tol=0.05,
                            coarse_maxiter=200, fine_prec="f64", coarse_prec="f64", squared=squared)
    # the 9-point setup adapts nvec / 2 vectors and adds their reflections; the squared one adapts all nvec
    mg.mgdwf_setup(h, prm, dev(random_starts(L, LS, nvec if squared else nvec // 2, 81)))
    v0 = gaussian_fermion(L, LS, 82)
    ev, vecs, res = mg.mgdwf_low_modes(h, dev(v0), nev, 48, solve_tol=1e-12)
    print("gpu", ev, "\ndense", lam[:nev], "\nresid", res, flush=True)
    assert np.all(np.abs(np.array(ev) - lam[:nev]) <= 1e-9 * lam[:nev])
    assert max(res) < 1e-6
    Y = vecs.cpu().numpy()
    for i in range(nev):
        gap = min(abs(lam[i] - lam[j]) for j in range(len(lam)) if j != i) / lam[i]
        if gap > 1e-3:  # a simple eigenvalue: the vector is fixed up to a phase
            assert abs(abs(np.vdot(E[i], Y[i])) - 1.0) < 1e-7, i
        # every Ritz vector lies in the oracle's lowest eigenspace
        proj = sum(abs(np.vdot(E[j], Y[i])) ** 2 for j in range(len(lam)))
        assert proj > 1 - 1e-8
    h.close()


def test_coverage_matches_oracle_and_low_mode_basis_covers_its_modes(cuda, dense):
    import paper_1205_2933_amd as mg
    U, lam, E = dense
    h = mg.Handle(L, LS, M5, MF)
    mg.mgdwf_set_gauge(h, dev(U))
    V = random_starts(L, LS, 6, 83)
    mg.mgdwf_set_nullvecs(h, BLOCK, dev(V), 6)
    Vh = torch.empty_like(dev(V))
    mg.mgdwf_get_basis(h, Vh)
    got = np.array(mg.mgdwf_coarse_coverage(h, dev(E), len(E)))
    want = olm.coverage(E, Vh.cpu().numpy(), BLOCK)
    assert np.abs(got - want).max() < 1e-12
    # Fig. 1's construction: the lowest four modes as the basis
    mg.mgdwf_set_nullvecs(h, BLOCK, dev(E[:4]), 4)
    got = np.array(mg.mgdwf_coarse_coverage(h, dev(E), len(E)))
    want = olm.coverage(E, ot.build_basis(E[:4], BLOCK), BLOCK)
    print("coverage by the 4-mode basis", np.round(got, 4), flush=True)
    assert np.allclose(got[:4], 1.0, atol=1e-12)
    assert np.abs(got - want).max() < 1e-12
    h.close()


def test_low_modes_arguments_are_validated(cuda, dense):
    import paper_1205_2933_amd as mg
    U = dense[0]
    h = mg.Handle(L, LS, M5, MF)
    mg.mgdwf_set_gauge(h, dev(U))
    v0 = dev(gaussian_fermion(L, LS, 84))
    with pytest.raises(mg.MgdwfError) as e:  # no multigrid yet
        mg.mgdwf_low_modes(h, v0, 4, 8)
    assert e.value.status == mg.MGDWF_ERR_STATE
    mg.mgdwf_setup(h, mg.make_mg_params(BLOCK, 4, fine_prec="f64", coarse_prec="f64"), dev(random_starts(L, LS, 2, 85)))
    for nev, m, tol in ((0, 8, 1e-10), (9, 8, 1e-10), (4, 300, 1e-10), (4, 8, 0.1)):
        with pytest.raises(mg.MgdwfError) as e:
            mg.mgdwf_low_modes(h, v0, nev, m, solve_tol=tol)
        assert e.value.status == mg.MGDWF_ERR_INVALID_ARG
    with pytest.raises(mg.MgdwfError):  # zero start vector
        mg.mgdwf_low_modes(h, torch.zeros_like(v0), 4, 8)
    h.close()
