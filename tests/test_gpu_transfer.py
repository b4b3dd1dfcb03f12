"""GPU parity of the transfer operators and the coarse operator against the oracle.

Paper Sec. 1 (R, P, R P = 1), Sec. 2 (blocks over all of Ls; chirality split),
Sec. 4 (the unsquared operator's coarse stencil: self + 8 neighbours).
The orthonormal basis is unique (thin QR with positive real diagonal), so the
GPU basis is compared with the oracle's within 1e-13 * kappa (panel condition
number); R, P and D_c are compared on the GPU's own basis within 1e-13.
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion, prepare_gauge, random_starts
from oracle import coarse as oc
from oracle import transfer as ot

pytestmark = pytest.mark.gpu

CASES = [
    # (L, Ls, block, nvec, mf, bc)
    ((4, 4, 4, 4), 8, (2, 2, 2, 2), 8, 0.01, (1, 1, 1, 1)),     # C1: coarse extent 2 (aliased +-mu)
    ((2, 2, 2, 2), 4, (2, 2, 2, 2), 6, 0.05, (1, 1, 1, 1)),     # a single coarse site: all d alias to self
    ((8, 4, 6, 4), 6, (4, 2, 2, 4), 10, 0.02, (1, -1, 1, -1)),  # ragged, coarse extents 2,2,3,1
    ((4, 4, 6, 6), 4, (2, 2, 2, 2), 16, 0.001, (1, 1, 1, 1)),   # coarse extent 3: true 9-point stencil
    ((4, 2, 6, 6), 4, (2, 2, 2, 3), 32, 0.01, (1, 1, -1, 1)),   # the largest coarse block (2 Nv = 64)
]

# 16-bit storage: per-block scale, FP32 accumulation.  Unit roundoff 2^-11 (FP16)
# and 2^-8 (BF16, round to nearest even) on every matrix and vector entry; with
# the per-site vector scale the relative error of y stays within a few units.
LOWP_TOL = {"f16": 3e-3, "bf16": 2.5e-2}


# per coarse site the relative error may exceed the global one where a site's
# output is smaller than average (measured: worst site 1.3x the global error
# in every precision); the bound allows 2x
SITE_FACTOR = 2.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def site_max_rel(got, want):
    """max over coarse sites of |got(X) - want(X)| / |want(X)| (all 2 Nv components of a site)."""
    g = got.reshape(-1, got.shape[-2] * got.shape[-1])
    w = want.reshape(g.shape)
    return float(np.max(np.linalg.norm(g - w, axis=1) / np.linalg.norm(w, axis=1)))


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def panel_kappa(V, block):
    A = ot._chiral_panels(V, block)
    s = np.linalg.svd(A, compute_uv=False)
    return float(np.max(s[..., 0] / s[..., -1]))


def make(case, mg):
    L, Ls, block, nvec, mf, bc = case
    U = prepare_gauge(L, 0.4, 31)
    V = random_starts(L, Ls, nvec, 41)
    h = mg.Handle(L, Ls, 1.8, mf, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    mg.mgdwf_set_nullvecs(h, block, dev(V), nvec)
    Vh = torch.empty_like(dev(V))
    mg.mgdwf_get_basis(h, Vh)
    torch.cuda.synchronize()
    return h, U, V, Vh.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_b{''.join(map(str, c[2]))}")
def test_basis_matches_oracle_qr(cuda, case):
    import paper_1205_2933_amd as mg
    print(f"basis case {case}", flush=True)
    h, U, V, Vh = make(case, mg)
    ref = ot.build_basis(V, case[2])
    kappa = panel_kappa(V, case[2])
    assert rel(Vh, ref) < 1e-13 * max(1.0, kappa)
    # orthonormal panels: P^+ P = 1 through the oracle's own restriction
    c = np.random.default_rng(0).standard_normal(ot.restrict(V[0], ref, case[2]).shape) + 0j
    assert rel(ot.restrict(ot.prolong(c, Vh, case[2]), Vh, case[2]), c) < 1e-13


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_b{''.join(map(str, c[2]))}")
def test_restrict_prolong_match_oracle(cuda, case):
    """R and P on 5 right-hand sides: the multi-RHS kernels read the basis once
    per group of right-hand sides, with a ragged last group."""
    import paper_1205_2933_amd as mg
    L, Ls, block, nvec, mf, bc = case
    h, U, V, Vh = make(case, mg)
    n = 5
    x = gaussian_fermion(L, Ls, 51, n=n)
    cshape = ot.restrict(x[0], Vh, block).shape
    cg = torch.empty((n,) + cshape, dtype=torch.complex128, device="cuda")
    mg.mgdwf_restrict(h, dev(x), cg, nrhs=n)
    c = np.random.default_rng(1).standard_normal((n,) + cshape) + 1j * np.random.default_rng(2).standard_normal((n,) + cshape)
    fg = torch.empty_like(dev(x))
    mg.mgdwf_prolong(h, dev(c), fg, nrhs=n)
    c1 = torch.empty((1,) + cshape, dtype=torch.complex128, device="cuda")
    mg.mgdwf_restrict(h, dev(x[3:4]), c1, nrhs=1)
    torch.cuda.synchronize()
    for r in range(n):
        assert rel(cg.cpu().numpy()[r], ot.restrict(x[r], Vh, block)) < 1e-13
        assert rel(fg.cpu().numpy()[r], ot.prolong(c[r], Vh, block)) < 1e-13
    assert rel(c1.cpu().numpy()[0], cg.cpu().numpy()[3]) < 1e-14


@pytest.mark.parametrize("n", [2, 13])
def test_restrict_prolong_fp32_kernels(cuda, n):
    """The V-cycle's FP32 R and P: 4^4 blocks put 1024 rows in each quarter
    block, so R takes the LDS-staged kernel (12 right-hand sides per group,
    13 leaves a group of one); FP32 rounding of basis and fields bounds the
    error at a few 1e-7 relative."""
    import paper_1205_2933_amd as mg
    case = ((8, 8, 8, 8), 4, (4, 4, 4, 4), 24, 0.01, (1, 1, 1, 1))
    L, Ls, block, nvec, mf, bc = case
    h, U, V, Vh = make(case, mg)
    x = gaussian_fermion(L, Ls, 61, n=n)
    cshape = ot.restrict(x[0], Vh, block).shape
    cg = torch.empty((n,) + cshape, dtype=torch.complex128, device="cuda")
    mg.mgdwf_restrict(h, dev(x), cg, nrhs=n, prec="f32")
    rng = np.random.default_rng(3)
    c = rng.standard_normal((n,) + cshape) + 1j * rng.standard_normal((n,) + cshape)
    fg = torch.empty_like(dev(x))
    mg.mgdwf_prolong(h, dev(c), fg, nrhs=n, prec="f32")
    torch.cuda.synchronize()
    for r in range(n):
        assert rel(cg.cpu().numpy()[r], ot.restrict(x[r], Vh, block)) < 1e-5
        assert rel(fg.cpu().numpy()[r], ot.prolong(c[r], Vh, block)) < 1e-5


def test_rank_deficient_basis_is_rejected(cuda):
    import paper_1205_2933_amd as mg
    L, Ls = (4, 4, 4, 4), 4
    U = prepare_gauge(L, 0.3, 1)
    V = random_starts(L, Ls, 4, 2)
    V[3] = V[1]  # duplicated vector -> dependent columns in every panel
    h = mg.Handle(L, Ls, 1.8, 0.01)
    mg.mgdwf_set_gauge(h, dev(U))
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_set_nullvecs(h, (2, 2, 2, 2), dev(V), 4)
    assert e.value.status == mg.MGDWF_ERR_NUMERIC


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_b{''.join(map(str, c[2]))}")
def test_coarse_operator_matches_oracle(cuda, case):
    import paper_1205_2933_amd as mg
    L, Ls, block, nvec, mf, bc = case
    h, U, V, Vh = make(case, mg)
    mg.mgdwf_build_coarse(h)
    Lc = tuple(L[m] // block[m] for m in range(4))
    n2 = 2 * nvec
    Dc = torch.empty(Lc[::-1] + (9, n2, n2), dtype=torch.complex128, device="cuda")
    mg.mgdwf_get_coarse_op(h, Dc)
    torch.cuda.synchronize()
    ref = oc.build_coarse_op(Vh, U, 1.8, mf, block, bc)
    assert rel(Dc.cpu().numpy(), ref) < 1e-13
    # apply, both directions, FP64 and FP32
    c = np.random.default_rng(3).standard_normal(Lc[::-1] + (2, nvec)) + 1j * np.random.default_rng(4).standard_normal(Lc[::-1] + (2, nvec))
    precs = [("f64", 1e-13, 0), ("f32", 2e-6, 0)]
    if nvec % 8 == 0:  # both MFMA shapes of the 16-bit apply
        precs += [(p, LOWP_TOL[p], ct) for p in ("f16", "bf16") for ct in (0, 1)]
    for dagger in (False, True):
        for prec, tol, ct in precs:
            mg.mgdwf_set_coarse_tiling(h, ct)
            y = torch.empty_like(dev(c))
            mg.mgdwf_apply_coarse(h, dev(c), y, dagger=dagger, prec=prec)
            torch.cuda.synchronize()
            got, want = y.cpu().numpy(), oc.apply_coarse(c, ref, dagger=dagger)
            assert rel(got, want) < tol, (dagger, prec, ct)
            # site by site: no single coarse site may hide a larger error
            worst = site_max_rel(got, want)
            print(f"{prec} ct={ct} dagger={dagger} global {rel(got, want):.2e} worst site {worst:.2e}", flush=True)
            assert worst < SITE_FACTOR * tol, (dagger, prec, ct, worst)
    mg.mgdwf_set_coarse_tiling(h, -1)
    with pytest.raises(mg.MgdwfError):
        mg.mgdwf_set_coarse_tiling(h, 2)


def test_coarse_apply_many_rhs(cuda):
    """18 right-hand sides: crosses the 8-RHS (FP64) and 16-RHS (FP32, MFMA) chunks."""
    import paper_1205_2933_amd as mg
    case = CASES[3]
    L, Ls, block, nvec, mf, bc = case
    h, U, V, Vh = make(case, mg)
    mg.mgdwf_build_coarse(h)
    Lc = tuple(L[m] // block[m] for m in range(4))
    ref = oc.build_coarse_op(Vh, U, 1.8, mf, block, bc)
    nr = 18
    rng = np.random.default_rng(9)
    c = rng.standard_normal((nr,) + Lc[::-1] + (2, nvec)) + 1j * rng.standard_normal((nr,) + Lc[::-1] + (2, nvec))
    c[5] *= 1e-6   # a small RHS next to O(1) ones: the per-(site, RHS) scale keeps it accurate
    for dagger in (False, True):
        want = np.stack([oc.apply_coarse(c[r], ref, dagger=dagger) for r in range(nr)])
        for prec, tol, ct in (("f64", 1e-13, 0), ("f32", 2e-6, 0), ("f16", LOWP_TOL["f16"], 0),
                              ("bf16", LOWP_TOL["bf16"], 0), ("f16", LOWP_TOL["f16"], 1),
                              ("bf16", LOWP_TOL["bf16"], 1)):
            mg.mgdwf_set_coarse_tiling(h, ct)
            y = torch.empty_like(dev(c))
            mg.mgdwf_apply_coarse(h, dev(c), y, dagger=dagger, prec=prec, nrhs=nr)
            torch.cuda.synchronize()
            got = y.cpu().numpy()
            for r in range(nr):
                assert rel(got[r], want[r]) < tol, (dagger, prec, ct, r)
                assert site_max_rel(got[r], want[r]) < SITE_FACTOR * tol, (dagger, prec, ct, r)
    # the tuner times both shapes once a coarse operator exists
    rep = mg.mgdwf_tune(h, nrhs=nr, iters=2)
    assert rep["coarse_chosen"] in (0, 1) and len(rep["coarse_us"]) == 2
    assert rep["coarse_chosen"] == 0 or rep["coarse_us"][1] <= 0.97 * rep["coarse_us"][0]
