"""GPU 2D U(1) model (the paper's Sec. 3 test problem, Fig. 2) against the
oracle, through the C ABI (mgdwf_create_2d):

* D and D^+ in FP64 (1e-13) and FP32 (2e-6) on 20^2 x 8 (antiperiodic y), on
  odd extents and on Ls = 1, several right-hand sides;
* the chirality-split block basis (1e-12), R and P (FP64 1e-13, FP32 1e-6);
* A_c = P^+ D^+D P: the 33-offset store holds the oracle's 9-offset stencil
  (1e-12) with every offset along z and t zero, on coarse extents 3 and 5;
  its FP64 / FP32 apply equals R D^+D P by the oracle on coarse extent 2;
* one V-cycle application (coarse CG fixed at 16 iterations) equal to the
  oracle's: FP64 1e-10, FP32 1e-5;
* the setup's near-null vectors (CG on D^+D v = 0) equal the oracle's (1e-8);
* multigrid solves at the paper's 20^2 x 8, 16 vectors, 4^2 x 8 blocks reach
  1e-10 against the oracle's D; the CGNE control's iteration count equals the
  oracle's to within one check interval;
* the 4D-only calls refuse a 2D handle.
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion2d, point_sources2d, quenched_u1_2d, random_starts2d
from oracle import solvers as sol
from oracle import u1_2d as o

pytestmark = pytest.mark.gpu

M5 = 1.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _handle(mg, L, Ls, mf, U, bc=(1, 1)):
    h = mg.Handle2D(L, Ls, M5, mf, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    return h


@pytest.mark.parametrize("L,Ls,bc,sweeps", [((20, 20), 8, (1, -1), 50), ((5, 3), 3, (-1, 1), 0),
                                            ((4, 6), 1, (1, 1), 5)])
def test_dslash_matches_oracle(cuda, L, Ls, bc, sweeps):
    import paper_1205_2933_amd as mg
    U = quenched_u1_2d(L, 4.0, 3, sweeps=sweeps)
    mf = 0.04
    h = _handle(mg, L, Ls, mf, U, bc)
    x = gaussian_fermion2d(L, Ls, 5, n=3)
    for dag in (False, True):
        want = np.array([o.apply_dwf2(v, U, M5, mf, bc, dag) for v in x])
        for prec, tol in (("f64", 1e-13), ("f32", 2e-6)):
            out = torch.empty_like(dev(x))
            mg.mgdwf_apply_dwf(h, dev(x), out, dagger=dag, prec=prec, nrhs=3)
            e = rel(out.cpu().numpy(), want)
            print(f"2D dslash L={L} Ls={Ls} dag={dag} {prec}: {e:.2e}", flush=True)
            assert e < tol
    h.close()


def test_basis_and_transfer_match_oracle(cuda):
    import paper_1205_2933_amd as mg
    L, Ls, block, nv = (12, 8), 4, (4, 2), 6
    U = quenched_u1_2d(L, 4.0, 4, sweeps=20)
    h = _handle(mg, L, Ls, 0.05, U)
    V = random_starts2d(L, Ls, nv, 6)
    mg.mgdwf_set_nullvecs(h, block + (1, 1), dev(V), nv)
    Vh = torch.empty_like(dev(V))
    mg.mgdwf_get_basis(h, Vh)
    Vref = o.build_basis2d(V, block)
    assert rel(Vh.cpu().numpy(), Vref) < 1e-12
    x = gaussian_fermion2d(L, Ls, 7, n=3)
    Lc = (L[1] // block[1], L[0] // block[0])
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        c = torch.empty((3,) + Lc + (2, nv), dtype=torch.complex128, device="cuda")
        mg.mgdwf_restrict(h, dev(x), c, nrhs=3, prec=prec)
        want = np.array([o.restrict2d(v, Vref, block) for v in x])
        assert rel(c.cpu().numpy(), want) < tol
        f = torch.empty_like(dev(x))
        mg.mgdwf_prolong(h, dev(want), f, nrhs=3, prec=prec)
        assert rel(f.cpu().numpy(), np.array([o.prolong2d(w, Vref, block) for w in want])) < tol
    h.close()


OFF9 = [0, 1, 2, 3, 4, 9, 10, 11, 12]  # the 2D offsets in the 33-offset order


@pytest.mark.parametrize("L,block", [((12, 12), (4, 4)), ((20, 10), (4, 2))])
def test_coarse_operator_matches_oracle(cuda, L, block):
    import paper_1205_2933_amd as mg
    Ls, nv, mf = 4, 4, 0.03
    U = quenched_u1_2d(L, 4.0, 8, sweeps=20)
    h = _handle(mg, L, Ls, mf, U, (1, -1))
    V = random_starts2d(L, Ls, nv, 9)
    mg.mgdwf_set_nullvecs(h, block + (1, 1), dev(V), nv)
    mg.mgdwf_build_coarse_squared(h)
    assert mg.mgdwf_coarse_stencil_size(h) == 33
    Yc, Xc = L[1] // block[1], L[0] // block[0]
    A = torch.empty((1, 1, Yc, Xc, 33, 2 * nv, 2 * nv), dtype=torch.complex128, device="cuda")
    mg.mgdwf_get_coarse_op(h, A)
    A = A.cpu().numpy()[0, 0]
    ref = o.build_sq_coarse_op2d(o.build_basis2d(V, block), U, M5, mf, block, (1, -1))
    assert np.abs(A[:, :, OFF9] - ref).max() < 1e-12 * np.abs(ref).max()
    rest = [k for k in range(33) if k not in OFF9]
    assert np.abs(A[:, :, rest]).max() == 0.0
    h.close()


def test_coarse_apply_on_extent_two(cuda):
    import paper_1205_2933_amd as mg
    L, Ls, block, nv, mf = (8, 8), 4, (4, 4), 3, 0.02
    U = quenched_u1_2d(L, 4.0, 10, sweeps=20)
    h = _handle(mg, L, Ls, mf, U)
    V = random_starts2d(L, Ls, nv, 11)
    mg.mgdwf_set_nullvecs(h, block + (1, 1), dev(V), nv)
    mg.mgdwf_build_coarse_squared(h)
    ex = o.ExplicitCoarse2D(o.DWF2(U, M5, mf), o.build_basis2d(V, block), block)
    rng = np.random.default_rng(2)
    c = rng.standard_normal((2, 2, 2, 2, nv)) + 1j * rng.standard_normal((2, 2, 2, 2, nv))
    want = np.array([ex(v) for v in c])
    for prec, tol in (("f64", 1e-13), ("f32", 2e-6)):
        y = torch.empty_like(dev(c))
        mg.mgdwf_apply_coarse(h, dev(c), y, prec=prec, nrhs=2)
        assert rel(y.cpu().numpy(), want) < tol
    h.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_vcycle_matches_oracle(cuda, prec, tol):
    import paper_1205_2933_amd as mg
    L, Ls, block, nv, mf = (12, 12), 4, (4, 4), 6, 0.02
    U = quenched_u1_2d(L, 4.0, 12, sweeps=30)
    h = _handle(mg, L, Ls, mf, U)
    V = random_starts2d(L, Ls, nv, 13)
    mg.mgdwf_set_nullvecs(h, block + (1, 1), dev(V), nv)
    mg.mgdwf_build_coarse_squared(h)
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block + (1, 1), nv, nu_pre=3, nu_post=2, coarse_tol=1e-30,
                                                coarse_maxiter=16, fine_prec=prec, coarse_prec=prec, squared=True))
    A = o.DWF2(U, M5, mf)
    Vh = o.build_basis2d(V, block)
    M = o.TwoLevelSquared2D(A, Vh, block, o.ExplicitCoarse2D(A, Vh, block), 1e-30, 16, 3, 2)
    b = gaussian_fermion2d(L, Ls, 14, n=2)
    z = torch.empty_like(dev(b))
    mg.mgdwf_apply_vcycle(h, dev(b), z, nrhs=2)
    for r in range(2):
        e = rel(z.cpu().numpy()[r], M(b[r]))
        print(f"2D V-cycle {prec} rhs {r}: {e:.2e}", flush=True)
        assert e < tol
    h.close()


def test_setup_vectors_match_oracle(cuda):
    import paper_1205_2933_amd as mg
    L, Ls, block, nv, mf = (8, 8), 4, (4, 4), 4, 0.05
    U = quenched_u1_2d(L, 4.0, 15, sweeps=30)
    h = _handle(mg, L, Ls, mf, U)
    V0 = random_starts2d(L, Ls, nv, 16)
    p = mg.make_mg_params(block + (1, 1), nv, sweeps=1, sweep0_iters=20, fine_prec="f64", coarse_prec="f64",
                          squared=True)
    mg.mgdwf_setup(h, p, dev(V0))
    got = mg.mgdwf_get_nullvecs(h).cpu().numpy()
    A = o.DWF2(U, M5, mf)
    from oracle import setup as osetup
    for k in range(nv):
        w = osetup.cgnr_null_steps(A, V0[k], 20)
        w = w / np.linalg.norm(w)
        assert rel(got[k], w) < 1e-8, k
    h.close()


@pytest.fixture(scope="module")
def paper_lattice():
    L, Ls = (20, 20), 8
    return L, Ls, quenched_u1_2d(L, 4.0, 7)


@pytest.mark.parametrize("fine", ["f64", "f32"])
def test_multigrid_solves_paper_lattice(cuda, paper_lattice, fine):
    import paper_1205_2933_amd as mg
    L, Ls, U = paper_lattice
    mf = 0.01
    h = _handle(mg, L, Ls, mf, U)
    p = mg.make_mg_params((4, 4, 1, 1), 16, sweeps=1, sweep0_iters=100, nu_pre=4, nu_post=4, coarse_tol=0.1,
                          coarse_maxiter=500, fine_prec=fine, coarse_prec=fine, squared=True)
    mg.mgdwf_setup(h, p, dev(random_starts2d(L, Ls, 16, 21)))
    b = point_sources2d(L, Ls)
    x = torch.zeros_like(dev(b))
    reps = mg.mgdwf_solve(h, dev(b), x, nrhs=2, tol=1e-10, max_outer=200, restart=8)
    xs = x.cpu().numpy()
    for r in range(2):
        assert rel(o.apply_dwf2(xs[r], U, M5, mf), b[r]) < 1e-10
    # the oracle on the GPU's basis: the same number of outer iterations to within 10 %
    Vh = torch.empty((16,) + (L[1], L[0], Ls, 2), dtype=torch.complex128, device="cuda")
    mg.mgdwf_get_basis(h, Vh)
    A = o.DWF2(U, M5, mf)
    mgo = o.U1MG(A, o.U1Params(block=(4, 4), nvec=16, nu_pre=4, nu_post=4, coarse_tol=0.1, coarse_maxiter=500))
    mgo.Vhat = Vh.cpu().numpy()
    mgo.coarse = o.ExplicitCoarse2D(A, mgo.Vhat, (4, 4))
    _, rep, _ = o.u1_solve(mgo, b[0], 1e-10, 200, 8)
    print(f"2D MG {fine}: GPU {reps[0]['outer_iters']} outer, oracle {rep.iters}", flush=True)
    assert rep.converged
    assert abs(reps[0]["outer_iters"] - rep.iters) <= max(2, rep.iters // 10)
    h.close()


def test_cgne_control_matches_oracle(cuda, paper_lattice):
    import paper_1205_2933_amd as mg
    L, Ls, U = paper_lattice
    mf = 0.05
    h = _handle(mg, L, Ls, mf, U)
    b = point_sources2d(L, Ls)[0]
    x = torch.zeros_like(dev(b))
    rep = mg.mgdwf_cgne(h, dev(b), x, tol=1e-8, max_iter=20000)
    assert rel(o.apply_dwf2(x.cpu().numpy(), U, M5, mf), b) < 1e-8
    _, orep = sol.cgne(o.DWF2(U, M5, mf), b, 1e-8, 20000)
    print(f"2D CGNE: GPU {rep['outer_iters']}, oracle {orep.iters}", flush=True)
    assert orep.iters <= rep["outer_iters"] <= orep.iters + 16  # the GPU tests every 16 iterations
    h.close()


def test_4d_only_calls_refuse_a_2d_handle(cuda):
    import paper_1205_2933_amd as mg
    L, Ls = (8, 8), 2
    h = _handle(mg, L, Ls, 0.1, quenched_u1_2d(L, 4.0, 1, sweeps=5))
    mg.mgdwf_set_nullvecs(h, (4, 4, 1, 1), dev(random_starts2d(L, Ls, 2, 3)), 2)
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_build_coarse(h)
    assert e.value.status == mg.MGDWF_ERR_INVALID_ARG
    with pytest.raises(mg.MgdwfError):
        mg.mgdwf_set_mg_params(h, mg.make_mg_params((4, 4, 1, 1), 2, squared=False))
    with pytest.raises(mg.MgdwfError):
        mg.mgdwf_tune(h, 1, 1)
    with pytest.raises(mg.MgdwfError):  # a block of 1 along x: no squared stencil
        mg.mgdwf_set_nullvecs(h, (1, 4, 1, 1), dev(random_starts2d(L, Ls, 2, 3)), 2)
        mg.mgdwf_build_coarse_squared(h)
    h.close()


def test_2d_checkpoint_reloads_bitwise(cuda, tmp_path):
    """A 2D setup saved and loaded into a fresh 2D handle solves bit for bit
    as the saved one; a 4D handle refuses the file."""
    import paper_1205_2933_amd as mg
    L, Ls, mf = (8, 8), 4, 0.05
    U = quenched_u1_2d(L, 4.0, 17, sweeps=20)
    h = _handle(mg, L, Ls, mf, U)
    p = mg.make_mg_params((4, 4, 1, 1), 4, sweeps=1, sweep0_iters=30, nu_pre=3, nu_post=3, coarse_tol=0.1,
                          fine_prec="f64", coarse_prec="f64", squared=True)
    mg.mgdwf_setup(h, p, dev(random_starts2d(L, Ls, 4, 18)))
    path = tmp_path / "u1.ck"
    mg.mgdwf_save_setup(h, path)
    b = dev(point_sources2d(L, Ls)[0])
    x0 = torch.zeros_like(b)
    mg.mgdwf_solve(h, b, x0, tol=1e-10, max_outer=200, restart=8)
    h2 = _handle(mg, L, Ls, mf, U)
    mg.mgdwf_load_setup(h2, path)
    mg.mgdwf_set_mg_params(h2, p)
    x1 = torch.zeros_like(b)
    mg.mgdwf_solve(h2, b, x1, tol=1e-10, max_outer=200, restart=8)
    assert torch.equal(x0, x1)
    h4 = mg.Handle((4, 4, 4, 4), Ls, M5, mf)
    with pytest.raises(mg.MgdwfError):
        mg.mgdwf_load_setup(h4, path)
    for hh in (h, h2, h4):
        hh.close()
