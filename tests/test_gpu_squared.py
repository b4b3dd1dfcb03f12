"""GPU squared-operator multigrid against the oracle (paper Sec. 3 first
paragraph: the multigrid acts on D^+D; Sec. 4: its coarse operator reaches
two hops).

* A_c = P^+ D^+D P: the GPU's 33-offset stencil equals the oracle's (read
  off column by column from the definition) at 1e-13, and its FP64 / FP32
  application equals R D^+D P applied by the oracle, with coarse extents 1,
  2 and 3;
* one V-cycle application (coarse CG fixed at 16 iterations on both sides)
  equals the oracle's: FP64 1e-10, FP32 1e-5;
* setup (sweep 0) null residual equals the oracle's at 1e-8;
* solves reach 1e-10 against the oracle's D, FP64 and mixed.
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion, prepare_gauge, random_starts
from oracle import dwf
from oracle import squared as osq
from oracle import transfer as ot

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _handle(mg, L, Ls, mf, block, nvec, seed, bc=(1, 1, 1, 1)):
    U = prepare_gauge(L, 0.4, seed)
    V = random_starts(L, Ls, nvec, seed + 1)
    h = mg.Handle(L, Ls, 1.8, mf, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    mg.mgdwf_set_nullvecs(h, block, dev(V), nvec)
    Vh = torch.empty_like(dev(V))
    mg.mgdwf_get_basis(h, Vh)
    mg.mgdwf_build_coarse_squared(h)
    return h, U, Vh.cpu().numpy()


def test_squared_stencil_matches_oracle(cuda):
    import paper_1205_2933_amd as mg
    L, Ls, mf, block, nvec = (6, 6, 6, 6), 2, 0.04, (2, 2, 2, 2), 2
    h, U, Vh = _handle(mg, L, Ls, mf, block, nvec, 50, bc=(1, -1, 1, 1))
    assert mg.mgdwf_coarse_stencil_size(h) == 33
    Lc = (3, 3, 3, 3)
    n2 = 2 * nvec
    Ac = torch.empty(Lc + (33, n2, n2), dtype=torch.complex128, device="cuda")
    mg.mgdwf_get_coarse_op(h, Ac)
    ref = osq.build_sq_coarse_op(Vh, U, 1.8, mf, block, (1, -1, 1, 1))
    assert rel(Ac.cpu().numpy(), ref) < 1e-13
    h.close()


@pytest.mark.parametrize("L,block,nvec", [((4, 4, 4, 4), (2, 2, 2, 2), 8),     # coarse extent 2: +-mu alias
                                          ((2, 4, 6, 4), (2, 2, 2, 2), 4),     # coarse extents 1, 2, 3
                                          ((8, 4, 6, 4), (4, 2, 2, 2), 16)])   # 4^1 blocks, 2 Nv = 32
def test_squared_apply_is_r_dd_p(cuda, L, block, nvec):
    import paper_1205_2933_amd as mg
    Ls, mf = 4, 0.02
    h, U, Vh = _handle(mg, L, Ls, mf, block, nvec, 52)
    A = dwf.DWF(U, 1.8, mf)
    Lc = tuple(L[m] // block[m] for m in range(4))
    # right-hand side counts that take every panel width of the apply
    # (FP64: 1, 4, 8 + 1; FP32: 1, 12, 16 + 2)
    for nr, prec, tol in ((1, "f64", 1e-12), (3, "f64", 1e-12), (9, "f64", 1e-12), (1, "f32", 2e-6),
                          (12, "f32", 2e-6), (18, "f32", 2e-6)):
        rng = np.random.default_rng(53)
        c = rng.standard_normal((nr,) + Lc[::-1] + (2, nvec)) + 1j * rng.standard_normal((nr,) + Lc[::-1] + (2, nvec))
        y = torch.empty_like(dev(c))
        mg.mgdwf_apply_coarse(h, dev(c), y, prec=prec, nrhs=nr)
        got = y.cpu().numpy()
        ex = osq.ExplicitCoarse(A, Vh, block)
        for r in range(nr):
            assert rel(got[r], ex(c[r])) < tol, (prec, r)
    h.close()


VTOL = {("f64", "f64"): 1e-10, ("f32", "f32"): 1e-5}


@pytest.mark.parametrize("prec,cprec", list(VTOL))
def test_squared_vcycle_matches_oracle(cuda, prec, cprec):
    """M(r) = V(D^+ r) with MR smoothing on D^+D (nu = 3 each), R, CG on
    A_c for 16 iterations, P, the residual recomputed with D^+D, post
    smoothing: the GPU's application equals the oracle's."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, block, nvec = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2), 8
    h, U, Vh = _handle(mg, L, Ls, mf, block, nvec, 54)
    A = dwf.DWF(U, 1.8, mf)
    M = osq.TwoLevelSquared(A, Vh, block, osq.ExplicitCoarse(A, Vh, block), 1e-30, 16, 3, 3)
    b = gaussian_fermion(L, Ls, 55, n=2)
    want = np.stack([M(b[r]) for r in range(2)])
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, nvec, nu_pre=3, nu_post=3, coarse_tol=1e-30,
                                                coarse_maxiter=16, fine_prec=prec, coarse_prec=cprec, squared=True))
    z = torch.empty_like(dev(b))
    mg.mgdwf_apply_vcycle(h, dev(b), z, nrhs=2)
    got = z.cpu().numpy()
    for r in range(2):
        e = rel(got[r], want[r])
        print(f"squared V-cycle {prec}/{cprec} rhs {r}: {e:.3e}", flush=True)
        assert e < VTOL[(prec, cprec)]
    h.close()


def test_squared_setup_and_solves(cuda):
    """Sweep 0 of the squared setup (8 vectors, CG on D^+D, no reflections)
    gives the oracle's median null residual; FP64 and mixed solves from that
    setup reach 1e-10 against the oracle's D, and the FP64 solve takes the
    oracle's number of outer iterations on the same basis (up to rounding)."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, block, nvec = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2), 16
    U = prepare_gauge(L, 0.3, 11)
    A = dwf.DWF(U, 1.8, mf)
    V0 = random_starts(L, Ls, nvec, 21)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    kw = dict(sweeps=1, sweep0_iters=100, nu_pre=4, nu_post=4, coarse_tol=0.1, coarse_maxiter=200, squared=True)
    rep = mg.mgdwf_setup(h, mg.make_mg_params(block, nvec, fine_prec="f64", coarse_prec="f64", **kw), dev(V0))
    prm = osq.SquaredParams(block=block, nvec=nvec, sweep0_iters=100, nu_pre=4, nu_post=4, coarse_tol=0.1,
                            coarse_maxiter=200)
    omg = osq.squared_setup(A, V0, prm)
    print("null residual gpu", rep["null_residual"], "oracle", omg.null_residuals, flush=True)
    assert abs(rep["null_residual"][0] - omg.null_residuals[0]) <= 1e-8 * omg.null_residuals[0]
    assert mg.mgdwf_coarse_stencil_size(h) == 33
    b = gaussian_fermion(L, Ls, 31)
    iters = {}
    for prec in ("f64", "f32"):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, nvec, fine_prec=prec, coarse_prec=prec, **kw))
        x = torch.zeros_like(dev(b))
        r = mg.mgdwf_solve(h, dev(b), x, tol=1e-10, max_outer=400, restart=8)[0]
        print("squared solve", prec, r, flush=True)
        xs = x.cpu().numpy()
        assert np.linalg.norm(b - dwf.apply_dwf(xs, U, 1.8, mf)) / np.linalg.norm(b) < 1e-10
        iters[prec] = r["outer_iters"]
        fine = r["fine_applies"]
    # the oracle's squared MG on the GPU's own basis (the coarse CG tests its
    # residual every iteration there, every 8 on the GPU: a few iterations apart)
    Vg = mg.mgdwf_get_nullvecs(h).cpu().numpy()
    omg.rebuild(Vg)
    _, orep = osq.squared_solve(omg, b, 1e-10, 400, 8)
    print("outer iterations gpu", iters, "oracle", orep.iters, flush=True)
    assert orep.converged
    assert abs(iters["f64"] - orep.iters) <= max(3, 0.1 * orep.iters)
    h.close()


def test_squared_params_are_validated(cuda):
    import paper_1205_2933_amd as mg
    L, Ls = (4, 4, 4, 4), 4
    h = mg.Handle(L, Ls, 1.8, 0.01)
    mg.mgdwf_set_gauge(h, dev(prepare_gauge(L, 0.3, 3)))
    V0 = dev(random_starts(L, Ls, 4, 4))
    with pytest.raises(mg.MgdwfError):  # 16-bit coarse level
        mg.mgdwf_setup(h, mg.make_mg_params((2, 2, 2, 2), 4, fine_prec="f32", coarse_prec="f16", squared=True), V0)
    with pytest.raises(mg.MgdwfError):  # a block of extent 1
        mg.mgdwf_setup(h, mg.make_mg_params((1, 2, 2, 2), 4, squared=True), V0)
    mg.mgdwf_set_nullvecs(h, (2, 2, 2, 2), V0, 4)
    mg.mgdwf_build_coarse(h)
    assert mg.mgdwf_coarse_stencil_size(h) == 9
    with pytest.raises(mg.MgdwfError) as e:  # squared parameters on the 9-point operator
        mg.mgdwf_set_mg_params(h, mg.make_mg_params((2, 2, 2, 2), 4, squared=True))
    assert e.value.status == mg.MGDWF_ERR_STATE
    h.close()
