"""The allocation-free application (edfa_apply_noalloc), through the C-ABI: two calls in a row
on different systems, the second smaller, each equal to edfa_apply on the same handle (the
same kernels on the same inputs, so bit for bit), FP64 and FP32, forward and transposed; a
system whose workspace exceeds the static array is refused with both sizes named, and so are a
transposed call before the transposed factors exist and a product whose SELL layout has not
been built yet."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu

KW = dict(variant="dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")


def _raw_noalloc(lib, P, r, z, transpose=0):
    L = lib.load()
    st = L.edfa_apply_noalloc(P._h, transpose, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_apply_on_two_calls(lib, precision):
    probs = [inputs.full_tensor_problem(12, sigma=2.0, corr=2.0, config_id=41),
             inputs.full_tensor_problem(7, 6, 5, sigma=2.0, corr=2.0, config_id=42)]
    for k, prob in enumerate(probs):
        S = lib.System(prob)
        P = lib.Precond(S, lib.Params(**KW, precision=precision))
        n = S.info["n"]
        r = torch.tensor(np.random.default_rng(k).standard_normal(n), device="cuda")
        ref = P.apply(r)                      # builds what the first application needs
        z = torch.full_like(r, float("nan"))
        assert _raw_noalloc(lib, P, r, z) == 0
        torch.cuda.synchronize()
        assert torch.equal(z, ref), (k, precision)
        reft = P.apply(r, transpose=True)
        zt = torch.full_like(r, float("nan"))
        assert _raw_noalloc(lib, P, r, zt, 1) == 0
        torch.cuda.synchronize()
        assert torch.equal(zt, reft), (k, precision)


def test_noalloc_refuses_what_it_would_have_to_allocate(lib):
    S = lib.System(inputs.full_tensor_problem(6, sigma=1.0, corr=1.0, config_id=43))
    P = lib.Precond(S, lib.Params(**KW))
    r = torch.ones(S.info["n"], dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    with pytest.raises(lib.EdfaError) as ei:
        P.apply(r, transpose=True, z=z, noalloc=True)
    assert "transposed factors" in str(ei.value)
    # a 96^3 grid needs more workspace than the static array holds
    big = lib.System(inputs.lognormal_iso_problem(96, config_id=44))
    Pb = lib.Precond(big, lib.Params("static"))
    rb = torch.ones(big.info["n"], dtype=torch.float64, device="cuda")
    with pytest.raises(lib.EdfaError) as ei:
        Pb.apply(rb, z=torch.empty_like(rb), noalloc=True)
    assert "bytes of workspace" in str(ei.value)
    # and the small handle still works afterwards
    zz = P.apply(r, noalloc=True)
    assert torch.equal(zz, P.apply(r))
    # the SELL layout of a long-row matrix (here M_L, whose default is the chunk kernel) is
    # built by its first product: refused until an application has run with it
    assert P.info()["chunks_ML"] > 0
    P.set_variant("sell/4", slot="M_L")
    with pytest.raises(lib.EdfaError) as ei:
        P.apply(r, z=z, noalloc=True)
    assert "SELL" in str(ei.value)
    ref = P.apply(r)
    assert torch.equal(P.apply(r, noalloc=True), ref)
    P.set_variant(None)
