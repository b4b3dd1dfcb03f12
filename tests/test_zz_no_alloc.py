"""The no-allocation coarse apply (mgdwf_apply_coarse_noalloc) against the
allocating one (mgdwf_apply_coarse), for callers that cannot allocate.

Both run the same kernels on the same inputs, so the outputs must be bitwise
equal; two calls in a row, the second with fewer right-hand sides, on the
9-point D_c (F64, F32, F16, BF16, both directions) and on the squared
operator's A_c (F64, F32).  A request beyond the 16 MiB scratch is refused.
"""
import numpy as np
import pytest
import torch

from inputs import prepare_gauge, random_starts

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _coarse_vec(Lc, nvec, nr, seed):
    rng = np.random.default_rng(seed)
    shp = (nr,) + tuple(Lc[::-1]) + (2, nvec)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


@pytest.mark.parametrize("squared", [False, True])
def test_noalloc_coarse_apply_equals_allocating_one(cuda, squared):
    import paper_1205_2933_amd as mg
    L, Ls, block, nvec = (4, 4, 4, 6), 4, (2, 2, 2, 2), 8
    Lc = tuple(L[m] // block[m] for m in range(4))
    h = mg.Handle(L, Ls, 1.8, 0.02)
    mg.mgdwf_set_gauge(h, dev(prepare_gauge(L, 0.4, 61)))
    mg.mgdwf_set_nullvecs(h, block, dev(random_starts(L, Ls, nvec, 62)), nvec)
    if squared:
        mg.mgdwf_build_coarse_squared(h)
        precs = ("f64", "f32")
    else:
        mg.mgdwf_build_coarse(h)
        precs = ("f64", "f32", "f16", "bf16")
    for prec in precs:
        for dagger in (False, True):
            for nr in (5, 2):  # the second call is smaller than the first
                c = dev(_coarse_vec(Lc, nvec, nr, 63 + nr))
                want = torch.empty_like(c)
                got = torch.full_like(c, float("nan"))
                mg.mgdwf_apply_coarse(h, c, want, dagger=dagger, prec=prec, nrhs=nr)
                mg.mgdwf_apply_coarse_noalloc(h, c, got, dagger=dagger, prec=prec, nrhs=nr)
                torch.cuda.synchronize()
                assert torch.equal(got, want), (squared, prec, dagger, nr)
    h.close()


def test_noalloc_refuses_more_than_its_scratch(cuda):
    import paper_1205_2933_amd as mg
    L, Ls, block, nvec = (4, 4, 4, 4), 2, (2, 2, 2, 2), 8
    h = mg.Handle(L, Ls, 1.8, 0.02)
    mg.mgdwf_set_gauge(h, dev(prepare_gauge(L, 0.4, 64)))
    mg.mgdwf_set_nullvecs(h, block, dev(random_starts(L, Ls, nvec, 65)), nvec)
    mg.mgdwf_build_coarse(h)
    nr = 4200  # 2 x 4200 x 16 sites x 16 dof x 8 B > 16 MiB
    c = torch.zeros((nr, 2, 2, 2, 2, 2, nvec), dtype=torch.complex128, device="cuda")
    out = torch.empty_like(c)
    with pytest.raises(mg.MgdwfError) as e:
        mg.mgdwf_apply_coarse_noalloc(h, c, out, prec="f32", nrhs=nr)
    assert e.value.status == mg.MGDWF_ERR_INVALID_ARG and "scratch" in str(e.value)
    mg.mgdwf_apply_coarse_noalloc(h, c, out, prec="f64", nrhs=nr)  # F64 needs no scratch
    h.close()
