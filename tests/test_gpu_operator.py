"""GPU parity of the fine operator (Dslash), through the C ABI, against the FP64 oracle.

Operator: the paper's Sec. 2 (fifth dimension) and Sec. 4 (one site plus ten
unit neighbours), Shamir form.  FP64 bar: relative error 1e-13; FP32: 2e-6
(single-precision rounding of ~30 accumulated terms).
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion, prepare_gauge
from oracle import dwf

pytestmark = pytest.mark.gpu

CASES = [
    # (L, Ls, eps, seed, mf, bc)
    ((4, 4, 4, 4), 8, 0.3, 11, 0.01, (1, 1, 1, 1)),       # C1 shape
    ((2, 2, 2, 2), 4, 0.6, 3, 0.1, (1, 1, 1, 1)),         # extent 2: x+mu == x-mu
    ((6, 4, 2, 8), 5, 0.5, 5, 0.05, (1, -1, 1, -1)),      # ragged extents, antiperiodic bc
    ((8, 6, 4, 4), 12, 0.4, 7, 0.001, (1, 1, 1, -1)),     # several workgroups + tail
    ((3, 3, 3, 3), 1, 0.4, 9, 0.2, (1, 1, 1, 1)),         # Ls = 1, odd extents
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}")
@pytest.mark.parametrize("dagger", [False, True])
def test_dslash_f64_matches_oracle(cuda, case, dagger):
    import paper_1205_2933_amd as mg
    L, Ls, eps, seed, mf, bc = case
    print(f"dslash f64 case L={L} Ls={Ls} dagger={dagger}", flush=True)
    U = prepare_gauge(L, eps, seed)
    psi = gaussian_fermion(L, Ls, seed + 100)
    h = mg.Handle(L, Ls, 1.8, mf, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    out = torch.empty_like(dev(psi))
    mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dagger, prec="f64")
    torch.cuda.synchronize()
    ref = dwf.apply_dwf(psi, U, 1.8, mf, bc, dagger=dagger)
    assert rel(out.cpu().numpy(), ref) < 1e-13


@pytest.mark.parametrize("case", CASES[:4], ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}")
def test_dslash_f32_matches_oracle(cuda, case):
    import paper_1205_2933_amd as mg
    L, Ls, eps, seed, mf, bc = case
    U = prepare_gauge(L, eps, seed)
    psi = gaussian_fermion(L, Ls, seed + 100)
    h = mg.Handle(L, Ls, 1.8, mf, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    for dagger in (False, True):
        out = torch.empty_like(dev(psi))
        mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dagger, prec="f32")
        torch.cuda.synchronize()
        ref = dwf.apply_dwf(psi, U, 1.8, mf, bc, dagger=dagger)
        assert rel(out.cpu().numpy(), ref) < 2e-6


def test_dslash_multi_rhs(cuda):
    import paper_1205_2933_amd as mg
    L, Ls = (4, 4, 4, 8), 8
    U = prepare_gauge(L, 0.3, 21)
    psi = gaussian_fermion(L, Ls, 22, n=3)
    h = mg.Handle(L, Ls, 1.8, 0.01)
    mg.mgdwf_set_gauge(h, dev(U))
    out = torch.empty_like(dev(psi))
    mg.mgdwf_apply_dwf(h, dev(psi), out, prec="f64", nrhs=3)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for r in range(3):
        assert rel(o[r], dwf.apply_dwf(psi[r], U, 1.8, 0.01)) < 1e-13


def test_dslash_deterministic(cuda):
    """Ten launches give bitwise identical results (no atomics, fixed order)."""
    import paper_1205_2933_amd as mg
    L, Ls = (4, 4, 4, 4), 8
    U = prepare_gauge(L, 0.3, 11)
    psi = dev(gaussian_fermion(L, Ls, 5))
    h = mg.Handle(L, Ls, 1.8, 0.01)
    mg.mgdwf_set_gauge(h, dev(U))
    outs = []
    for _ in range(10):
        o = torch.empty_like(psi)
        mg.mgdwf_apply_dwf(h, psi, o)
        outs.append(o)
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


def test_dslash_f32_every_tiling(cuda):
    """Each FP32 t-march tiling the autotuner may pick gives the operator; with
    t extent 7 the tilings that split t into chunks of 2 leave a short last one."""
    import paper_1205_2933_amd as mg
    L, Ls, mf, bc = (16, 16, 8, 7), 4, 0.02, (1, 1, -1, -1)
    U = prepare_gauge(L, 0.4, 31)
    psi = gaussian_fermion(L, Ls, 32, n=2)
    h = mg.Handle(L, Ls, 1.8, mf, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    rep = mg.mgdwf_tune(h, nrhs=2, iters=1)
    assert len(rep["id"]) >= 8 and 0 <= rep["chosen"] < len(rep["id"])
    assert any(t[3] == 2 for t in rep["tile"])
    assert {f for f in rep["flags"]} >= {0, 1, 2, 4, 12, 16, 20}
    # a tiling replaces the default only when at least 3 % faster
    c = rep["chosen"]
    assert c == 0 or rep["us"][c] <= 0.97 * rep["us"][0]
    refs = {dg: [dwf.apply_dwf(psi[r], U, 1.8, mf, bc, dagger=dg) for r in range(2)] for dg in (False, True)}
    for tid, tile in zip(rep["id"], rep["tile"]):
        print(f"tiling {tid} {tile}", flush=True)
        mg.mgdwf_set_tiling(h, tid)
        for dg in (False, True):
            out = torch.empty_like(dev(psi))
            mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dg, prec="f32", nrhs=2)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            for r in range(2):
                assert rel(o[r], refs[dg][r]) < 2e-6, (tid, tile, dg, r)
    with pytest.raises(mg.MgdwfError):
        mg.mgdwf_set_tiling(h, 10 ** 6)
    mg.mgdwf_set_tiling(h, -1)


@pytest.mark.parametrize("dagger", [False, True])
def test_dslash_f32_production_launch_ls16(cuda, dagger):
    """The FP32 launch the production solve uses: Ls = 16 on the default
    t-march tiling (4x4x2 sites per workgroup, 8 threads per 4D site), two
    right-hand sides, against the FP64 oracle at the FP32 bar."""
    import paper_1205_2933_amd as mg
    L, Ls, mf = (8, 8, 4, 4), 16, 0.001
    U = prepare_gauge(L, 0.3, 12, ape_steps=2)
    psi = gaussian_fermion(L, Ls, 77, n=2)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    out = torch.empty_like(dev(psi))
    mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dagger, prec="f32", nrhs=2)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for r in range(2):
        assert rel(o[r], dwf.apply_dwf(psi[r], U, 1.8, mf, dagger=dagger)) < 2e-6


def _integer_inputs(L, Ls, seed, n=1):
    """Links and fields with small Gaussian-integer entries (re, im in -2..2)."""
    rng = np.random.default_rng(seed)
    from inputs import fermion_shape, gauge_shape
    U = rng.integers(-1, 2, gauge_shape(L)) + 1j * rng.integers(-1, 2, gauge_shape(L))
    shp = ((n,) if n > 1 else ()) + fermion_shape(L, Ls)
    psi = rng.integers(-2, 3, shp) + 1j * rng.integers(-2, 3, shp)
    return U.astype(np.complex128), psi.astype(np.complex128)


@pytest.mark.parametrize("case", [((4, 4, 4, 4), 8, (1, 1, 1, 1)), ((2, 2, 2, 2), 4, (1, 1, 1, 1)),
                                  ((6, 4, 2, 8), 5, (1, -1, 1, -1)), ((8, 8, 4, 4), 16, (1, 1, 1, -1))],
                         ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}")
def test_dslash_integer_inputs_are_bit_exact(cuda, case):
    """Site and neighbour indexing, bit for bit: with Gaussian-integer links and
    fields, M5 = 1 and m_f = 1/2 every intermediate of D (and D^+) is a small
    dyadic number, exact in FP64 and FP32 whatever the summation order, so the
    GPU output must equal the oracle's exactly (extent 2, where x+mu == x-mu
    and both hops apply, included)."""
    import paper_1205_2933_amd as mg
    L, Ls, bc = case
    U, psi = _integer_inputs(L, Ls, 5, n=2)
    h = mg.Handle(L, Ls, 1.0, 0.5, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    for prec in ("f64", "f32"):
        for dagger in (False, True):
            out = torch.empty_like(dev(psi))
            mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dagger, prec=prec, nrhs=2)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            for r in range(2):
                ref = dwf.apply_dwf(psi[r], U, 1.0, 0.5, bc, dagger=dagger)
                assert np.array_equal(o[r], ref), (prec, dagger, r, np.abs(o[r] - ref).max())


@pytest.mark.parametrize("case", [((8, 8, 4, 6), 16, 5, (1, -1, 1, -1)), ((8, 4, 4, 5), 8, 11, (1, 1, -1, 1)),
                                  ((8, 8, 8, 4), 16, 12, (1, 1, 1, 1))],
                         ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}_n{c[2]}")
def test_dslash_f32_site_pair_tilings(cuda, case):
    """The wavefront-per-site-pair FP32 kernel (two x-neighbouring sites, R =
    32 / (Ls / 2) right-hand sides and all Ls per wavefront, links loaded once
    per site pair and broadcast across lanes, s-neighbours from neighbouring
    lanes) on every brick / t-chunk it admits, D and D^+, against the oracle:
    a ragged right-hand-side group (5 = 4 + 1 at Ls = 16, 11 = 8 + 3 at Ls = 8),
    odd t extents (short last chunk), antiperiodic directions, and the
    production 12 right-hand sides."""
    import paper_1205_2933_amd as mg
    L, Ls, nrhs, bc = case
    U = prepare_gauge(L, 0.4, 41)
    psi = gaussian_fermion(L, Ls, 42, n=nrhs)
    h = mg.Handle(L, Ls, 1.8, 0.01, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    rep = mg.mgdwf_tune(h, nrhs=nrhs, iters=1)
    ws = [(tid, tile) for tid, tile, fl in zip(rep["id"], rep["tile"], rep["flags"]) if fl & 32]
    assert len(ws) >= 2, rep
    refs = {dg: [dwf.apply_dwf(psi[r], U, 1.8, 0.01, bc, dagger=dg) for r in range(nrhs)] for dg in (False, True)}
    for tid, tile in ws:
        print(f"site-pair tiling {tid} {tile}", flush=True)
        mg.mgdwf_set_tiling(h, tid)
        for dg in (False, True):
            out = torch.empty_like(dev(psi))
            mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dg, prec="f32", nrhs=nrhs)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            for r in range(nrhs):
                assert rel(o[r], refs[dg][r]) < 2e-6, (tid, tile, dg, r)
    mg.mgdwf_set_tiling(h, -1)
    h.close()


def test_dslash_f32_site_pair_in_the_solver(cuda):
    """The site-pair kernel's residual mode (b - D x) and its per-RHS norms,
    as the V-cycle uses them: one mixed-precision V-cycle application with the
    site-pair tiling equals the one with the default tiling up to FP32
    rounding, and a solve with it reaches 1e-10 against the oracle's D."""
    import paper_1205_2933_amd as mg
    from inputs import random_starts
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    p = mg.make_mg_params(block, 16, sweeps=1, sweep0_iters=100, coarse_tol=1e-30, coarse_maxiter=16,
                          fine_prec="f32", coarse_prec="f32")
    mg.mgdwf_setup(h, p, dev(random_starts(L, Ls, 8, 21)))
    b = dev(gaussian_fermion(L, Ls, 31, n=3))
    z0 = torch.empty_like(b)
    mg.mgdwf_apply_vcycle(h, b, z0, nrhs=3)
    rep = mg.mgdwf_tune(h, nrhs=3, iters=1)
    ws = [tid for tid, fl in zip(rep["id"], rep["flags"]) if fl & 32]
    assert ws
    mg.mgdwf_set_tiling(h, ws[0])
    z1 = torch.empty_like(b)
    mg.mgdwf_apply_vcycle(h, b, z1, nrhs=3)
    e = float(torch.linalg.norm(z1 - z0) / torch.linalg.norm(z0))
    print("V-cycle site-pair vs default tiling", e, flush=True)
    assert e < 1e-5
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_tol=0.1, coarse_maxiter=200, fine_prec="f32",
                                                coarse_prec="f16"))
    x = torch.zeros_like(b)
    reps = mg.mgdwf_solve(h, b, x, nrhs=3, tol=1e-10, max_outer=400, restart=8)
    xs, bs = x.cpu().numpy(), b.cpu().numpy()
    for r in range(3):
        assert np.linalg.norm(bs[r] - dwf.apply_dwf(xs[r], U, 1.8, mf)) / np.linalg.norm(bs[r]) < 1e-10
    h.close()


@pytest.mark.parametrize("case", [((8, 8, 4, 6), 16, 3, (1, -1, 1, -1)), ((8, 4, 4, 5), 8, 2, (1, 1, -1, 1)),
                                  ((4, 4, 2, 3), 16, 2, (-1, 1, 1, -1)), ((16, 16, 16, 8), 16, 12, (1, 1, 1, -1))],
                         ids=lambda c: f"L{'x'.join(map(str, c[0]))}_Ls{c[1]}_n{c[2]}")
def test_dslash_f32_lds_exchange_tilings(cuda, case):
    """The FP32 t-march that keeps its tile's slice, links (phases folded in)
    and fifth-dimension neighbours in LDS and loads only face neighbours from
    memory, on every tile / t-chunk it admits, D and D^+, against the oracle:
    odd t extents (short last chunk), antiperiodic directions, a tile as wide
    as the lattice (4 x 4 x 2 on 4 x 4 x 2 x 3: every face neighbour wraps),
    and the production 12 right-hand sides at Ls = 16."""
    import paper_1205_2933_amd as mg
    L, Ls, nrhs, bc = case
    U = prepare_gauge(L, 0.4, 43)
    psi = gaussian_fermion(L, Ls, 44, n=nrhs)
    h = mg.Handle(L, Ls, 1.8, 0.01, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    rep = mg.mgdwf_tune(h, nrhs=nrhs, iters=1)
    tx = [(tid, tile) for tid, tile, fl in zip(rep["id"], rep["tile"], rep["flags"]) if fl & 64]
    assert tx, rep
    refs = {dg: [dwf.apply_dwf(psi[r], U, 1.8, 0.01, bc, dagger=dg) for r in range(nrhs)] for dg in (False, True)}
    for tid, tile in tx:
        print(f"LDS-exchange tiling {tid} {tile}", flush=True)
        mg.mgdwf_set_tiling(h, tid)
        for dg in (False, True):
            out = torch.empty_like(dev(psi))
            mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dg, prec="f32", nrhs=nrhs)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            for r in range(nrhs):
                assert rel(o[r], refs[dg][r]) < 2e-6, (tid, tile, dg, r)
    mg.mgdwf_set_tiling(h, -1)
    h.close()


def test_dslash_lds_exchange_integer_inputs_are_bit_exact(cuda):
    """Indexing of the LDS-exchange kernel bit for bit (Gaussian-integer links
    and fields, M5 = 1, m_f = 1/2, antiperiodic t and z): every tile it admits
    on 8 x 8 x 4 x 4 x 16 gives exactly the oracle's D and D^+."""
    import paper_1205_2933_amd as mg
    L, Ls, bc = (8, 8, 4, 4), 16, (1, 1, -1, -1)
    U, psi = _integer_inputs(L, Ls, 6, n=2)
    h = mg.Handle(L, Ls, 1.0, 0.5, bc)
    mg.mgdwf_set_gauge(h, dev(U))
    rep = mg.mgdwf_tune(h, nrhs=2, iters=1)
    tx = [tid for tid, fl in zip(rep["id"], rep["flags"]) if fl & 64]
    assert len(tx) >= 3
    refs = {dg: [dwf.apply_dwf(psi[r], U, 1.0, 0.5, bc, dagger=dg) for r in range(2)] for dg in (False, True)}
    for tid in tx:
        mg.mgdwf_set_tiling(h, tid)
        for dg in (False, True):
            out = torch.empty_like(dev(psi))
            mg.mgdwf_apply_dwf(h, dev(psi), out, dagger=dg, prec="f32", nrhs=2)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            for r in range(2):
                assert np.array_equal(o[r], refs[dg][r]), (tid, dg, r)
    h.close()


def test_dslash_lds_exchange_in_the_solver(cuda):
    """The LDS-exchange kernel's residual mode (b - D x) and per-RHS norms as
    the V-cycle uses them: one mixed-precision V-cycle application with it
    equals the default tiling's up to FP32 rounding, and a solve with it
    reaches 1e-10 against the oracle's D."""
    import paper_1205_2933_amd as mg
    from inputs import random_starts
    L, Ls, mf, block = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2)
    U = prepare_gauge(L, 0.3, 11)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    p = mg.make_mg_params(block, 16, sweeps=1, sweep0_iters=100, coarse_tol=1e-30, coarse_maxiter=16,
                          fine_prec="f32", coarse_prec="f32")
    mg.mgdwf_setup(h, p, dev(random_starts(L, Ls, 8, 21)))
    b = dev(gaussian_fermion(L, Ls, 31, n=3))
    z0 = torch.empty_like(b)
    mg.mgdwf_set_tiling(h, -1)
    mg.mgdwf_apply_vcycle(h, b, z0, nrhs=3)
    rep = mg.mgdwf_tune(h, nrhs=3, iters=1)
    tx = [tid for tid, fl in zip(rep["id"], rep["flags"]) if fl & 64]
    assert tx
    mg.mgdwf_set_tiling(h, tx[0])
    z1 = torch.empty_like(b)
    mg.mgdwf_apply_vcycle(h, b, z1, nrhs=3)
    e = float(torch.linalg.norm(z1 - z0) / torch.linalg.norm(z0))
    print("V-cycle LDS-exchange vs default tiling", e, flush=True)
    assert e < 1e-5
    mg.mgdwf_set_mg_params(h, mg.make_mg_params(block, 16, coarse_tol=0.1, coarse_maxiter=200, fine_prec="f32",
                                                coarse_prec="f16"))
    x = torch.zeros_like(b)
    reps = mg.mgdwf_solve(h, b, x, nrhs=3, tol=1e-10, max_outer=400, restart=8)
    xs, bs = x.cpu().numpy(), b.cpu().numpy()
    for r in range(3):
        assert reps[r]["true_relres"] < 1e-10
        assert np.linalg.norm(bs[r] - dwf.apply_dwf(xs[r], U, 1.8, mf)) / np.linalg.norm(bs[r]) < 1e-10
    h.close()
