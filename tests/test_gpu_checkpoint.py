"""Setup checkpoints through the C ABI (mgdwf_save_setup / mgdwf_load_setup).

A saved setup reloaded into a fresh handle on the same gauge field gives the
same basis and coarse operator bit for bit, and a solve from it repeats the
saved handle's solve exactly (9-point and squared operators); a file taken on
another gauge field or lattice is refused with MGDWF_ERR_STATE, a file that
is not a checkpoint with MGDWF_ERR_INVALID_ARG.
"""
import numpy as np
import pytest
import torch

from inputs import gaussian_fermion, prepare_gauge, random_starts

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("squared", [False, True])
def test_saved_setup_reloads_bitwise(cuda, tmp_path, squared):
    import paper_1205_2933_amd as mg
    L, Ls, mf, block, nvec = (4, 4, 4, 4), 8, 0.01, (2, 2, 2, 2), 16
    U = prepare_gauge(L, 0.3, 11)
    kw = dict(sweeps=1, sweep0_iters=60, coarse_tol=0.1, coarse_maxiter=200, fine_prec="f64", coarse_prec="f64",
              squared=squared)
    h = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h, dev(U))
    mg.mgdwf_setup(h, mg.make_mg_params(block, nvec, **kw), dev(random_starts(L, Ls, nvec if squared else nvec // 2, 21)))
    path = tmp_path / "setup.ck"
    mg.mgdwf_save_setup(h, path)
    b = dev(gaussian_fermion(L, Ls, 31))
    x0 = torch.zeros_like(b)
    r0 = mg.mgdwf_solve(h, b, x0, tol=1e-10, max_outer=400, restart=8)[0]
    Vh0 = torch.empty((nvec,) + b.shape, dtype=torch.complex128, device="cuda")
    mg.mgdwf_get_basis(h, Vh0)
    h2 = mg.Handle(L, Ls, 1.8, mf)
    mg.mgdwf_set_gauge(h2, dev(U))
    mg.mgdwf_load_setup(h2, path)
    assert h2.nvec == nvec and h2.block == block
    assert mg.mgdwf_coarse_stencil_size(h2) == (33 if squared else 9)
    Vh1 = torch.empty_like(Vh0)
    mg.mgdwf_get_basis(h2, Vh1)
    assert torch.equal(Vh0, Vh1)
    assert torch.equal(mg.mgdwf_get_nullvecs(h), mg.mgdwf_get_nullvecs(h2))
    with pytest.raises(mg.MgdwfError) as e:  # parameters are cleared by a load
        mg.mgdwf_solve(h2, b, torch.zeros_like(b), tol=1e-10)
    assert e.value.status == mg.MGDWF_ERR_STATE
    mg.mgdwf_set_mg_params(h2, mg.make_mg_params(block, nvec, **kw))
    x1 = torch.zeros_like(b)
    r1 = mg.mgdwf_solve(h2, b, x1, tol=1e-10, max_outer=400, restart=8)[0]
    assert r1["outer_iters"] == r0["outer_iters"]
    assert torch.equal(x0, x1)
    h.close()
    h2.close()


def test_checkpoint_refuses_other_fields_and_files(cuda, tmp_path):
    import paper_1205_2933_amd as mg
    L, Ls, block = (4, 4, 4, 4), 4, (2, 2, 2, 2)
    h = mg.Handle(L, Ls, 1.8, 0.01)
    mg.mgdwf_set_gauge(h, dev(prepare_gauge(L, 0.3, 3)))
    with pytest.raises(mg.MgdwfError) as e:  # nothing to save yet
        mg.mgdwf_save_setup(h, tmp_path / "none.ck")
    assert e.value.status == mg.MGDWF_ERR_STATE
    mg.mgdwf_set_nullvecs(h, block, dev(random_starts(L, Ls, 4, 4)), 4)
    mg.mgdwf_build_coarse(h)
    path = tmp_path / "a.ck"
    mg.mgdwf_save_setup(h, path)
    other = mg.Handle(L, Ls, 1.8, 0.01)
    mg.mgdwf_set_gauge(other, dev(prepare_gauge(L, 0.3, 4)))  # another gauge field
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_load_setup(other, path)
    assert e.value.status == mg.MGDWF_ERR_STATE
    mass = mg.Handle(L, Ls, 1.8, 0.02)  # another action
    mg.mgdwf_set_gauge(mass, dev(prepare_gauge(L, 0.3, 3)))
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_load_setup(mass, path)
    assert e.value.status == mg.MGDWF_ERR_STATE
    junk = tmp_path / "junk.ck"
    junk.write_bytes(b"not a checkpoint at all, just some bytes" * 4)
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_load_setup(h, junk)
    assert e.value.status == mg.MGDWF_ERR_INVALID_ARG
    trunc = tmp_path / "trunc.ck"
    trunc.write_bytes(path.read_bytes()[: 200 + path.stat().st_size // 2])
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_load_setup(h, trunc)
    assert e.value.status == mg.MGDWF_ERR_INVALID_ARG
    for x in (h, other, mass):
        x.close()
