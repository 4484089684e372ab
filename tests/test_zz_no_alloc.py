"""The build that allocates nothing (esmf_fock_build_noalloc) through the C
ABI: its workspace is the library's static device scratch.  Two calls in a
row, the second with a smaller molecule, each equal bitwise to
esmf_fock_build on the same handle and within the FP64 tolerance of the
oracle; a build whose workspace exceeds the scratch is refused before
anything is enqueued."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from gpu_util import announce, dev, host, maxabs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def pa():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2002_00322_amd as pa
    return pa


def _noalloc(pa, st, d, j, k, prec):
    from paper_2002_00322_amd import _native as nat
    import torch
    s = torch.cuda.current_stream()
    return nat.lib().esmf_fock_build_noalloc(st.handle, int(d.shape[0]), ctypes.c_void_p(d.data_ptr()),
                                             ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(k.data_ptr()),
                                             int(prec), ctypes.c_void_p(int(s.cuda_stream)))


def test_noalloc_build_equals_build_twice(pa, oracle_mod):
    import torch
    from paper_2002_00322_amd import _native as nat
    A, al = wl.chain(100)
    c_big = dict(name="chain200", centers=A, alpha=al, tau=1e-10, D=wl.transition_densities(200, 8, 40, 11, 12))
    c_small = wl.config1()   # box40, m = 4: the second call is smaller
    for c in (c_big, c_small):
        announce(f"noalloc build: {c['name']}")
        st = pa.EriStore(c["centers"], c["alpha"], c["tau"])
        d = dev(c["D"])
        j0, k0 = pa.fock_build(st, d)
        j1, k1 = torch.full_like(d, float("nan")), torch.full_like(d, float("nan"))
        torch.cuda.synchronize()
        assert _noalloc(pa, st, d, j1, k1, pa.PREC_FP64) == nat.ESMF_OK, nat.lib().esmf_last_error()
        torch.cuda.synchronize()
        assert torch.equal(j0, j1) and torch.equal(k0, k1)
        Jr, Kr = oracle_mod.jk_canonical(c["centers"], c["alpha"], c["tau"], c["D"])
        assert maxabs(host(j1), Jr) < TOL64 and maxabs(host(k1), Kr) < TOL64
        st.release()


def test_noalloc_refuses_a_workspace_beyond_the_scratch(pa):
    import torch
    from paper_2002_00322_amd import _native as nat
    A, al = wl.chain(300)   # chain600: about 600 MiB of workspace for m = 8
    st = pa.EriStore(A, al, 1e-10)
    assert st.info()["workspace_bytes"] > 256 << 20
    d = dev(wl.transition_densities(600, 8, 40, 13, 14))
    j, k = torch.full_like(d, 7.0), torch.full_like(d, 7.0)
    torch.cuda.synchronize()
    assert _noalloc(pa, st, d, j, k, pa.PREC_FP64) == nat.ESMF_ERR_INVALID_ARG
    assert b"scratch" in nat.lib().esmf_last_error()
    torch.cuda.synchronize()
    assert bool((j == 7.0).all()) and bool((k == 7.0).all())
    st.release()
