"""The allocation-free mobility apply (static device scratch) against the apply with a
caller workspace, through the C-ABI: two calls in a row, the second with a smaller input
(the scratch keeps the first call's contents), in both precisions, bitwise equal; and the
refusal of a size whose workspace exceeds the static array."""
import ctypes

import numpy as np
import pytest

from paper_1903_12609_amd import synth

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_apply_equals_workspace_apply(prec):
    import torch
    from paper_1903_12609_amd._native import lib, check, FilError
    L = lib()
    st = torch.cuda.current_stream().cuda_stream
    for S, a, eta in ((32000, 1.0, 1.0), (1037, 0.8, 1.7)):
        print("case noalloc prec", prec, "S", S, flush=True)
        Y, F, T = synth.rpy_throughput_inputs(S, seed=S)
        Yd, Fd, Td = _dev(Y), _dev(F), _dev(T)
        V0, W0 = torch.empty_like(Yd), torch.empty_like(Yd)
        V1, W1 = torch.full_like(Yd, float("nan")), torch.full_like(Yd, float("nan"))
        nb = int(L.fil_rpy_workspace_bytes(S, prec))
        assert 0 < nb <= int(L.fil_rpy_noalloc_scratch_bytes())
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        check(L.fil_rpy_mobility_apply(S, Yd.data_ptr(), Fd.data_ptr(), Td.data_ptr(), a, eta, prec, V0.data_ptr(),
                                       W0.data_ptr(), work.data_ptr(), nb, st))
        check(L.fil_rpy_mobility_apply_noalloc(S, Yd.data_ptr(), Fd.data_ptr(), Td.data_ptr(), a, eta, prec,
                                               V1.data_ptr(), W1.data_ptr(), st))
        torch.cuda.synchronize()
        assert torch.equal(V0, V1) and torch.equal(W0, W1)
    # a size whose workspace exceeds the static array is refused before anything runs
    big = 10_000_000  # its workspace exceeds the static array in both precisions
    assert int(L.fil_rpy_workspace_bytes(big, prec)) > int(L.fil_rpy_noalloc_scratch_bytes())
    p = ctypes.c_void_p(Yd.data_ptr())
    q = ctypes.c_void_p(V1.data_ptr())
    r = ctypes.c_void_p(W1.data_ptr())
    rc = L.fil_rpy_mobility_apply_noalloc(big, p, p, p, 1.0, 1.0, prec, q, r, st)
    assert rc == -1 and b"scratch" in L.fil_last_error()
