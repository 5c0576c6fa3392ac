"""rcqr_factor_static (the allocation-free entry point) through the C ABI, against rcqr_factor on
a plan: bitwise the same Q, R and status on two calls in a row, the second with a smaller input
(the static workspace keeps the first call's contents), plus the size limit and a failing input."""

import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


def plan_result(V, s1, s2, seed):
    m, n = V.shape
    with rc.Plan(m, n, s1, s2, seed) as p:
        Q, R = p.factor(V, check=False)
        st = p.info()
    return Q, R, st


def static_call(V, s1, s2, seed, Q=None):
    m, n = V.shape
    Q = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda") if Q is None else Q
    R = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    info = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    st = rc.lib().rcqr_factor_static(m, n, s1, s2, seed, 0, ctypes.c_void_p(V.data_ptr()), V.stride(0),
                                     ctypes.c_void_p(Q.data_ptr()), Q.stride(0), ctypes.c_void_p(R.data_ptr()), R.stride(0),
                                     ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    assert st == rc.OK
    torch.cuda.synchronize()
    return Q, R, tuple(int(x) for x in info.cpu())


def test_static_matches_plan_twice_smaller_second():
    cases = [(200_001, 64, 8192, 256, 1e10, 7), (10_000, 16, 512, 64, 1e4, 8)]
    for m, n, s1, s2, kappa, seed in cases:
        print("static entry point:", m, n, s1, s2, flush=True)
        V = torch.from_numpy(synth.make_V(m, n, kappa, seed)).to("cuda")
        Qp, Rp, stp = plan_result(V, s1, s2, seed)
        Qs, Rs, sts = static_call(V, s1, s2, seed)
        assert stp == (rc.OK, 0) and sts == stp
        assert torch.equal(Qs, Qp) and torch.equal(Rs, Rp)


def test_static_in_place_and_failure_status():
    m, n, s1, s2, seed = 30_000, 32, 2048, 128, 9
    Vh = synth.make_V(m, n, 1e6, seed)
    V = torch.from_numpy(Vh).to("cuda")
    Qp, Rp, _ = plan_result(V, s1, s2, seed)
    Vi = V.clone()
    Qi, Ri, st = static_call(Vi, s1, s2, seed, Q=Vi)
    assert st == (rc.OK, 0) and torch.equal(Qi, Qp) and torch.equal(Ri, Rp)
    Vz = V.clone()
    Vz[:, 5] = 0.0  # rank deficient: the sketch's R0 has a zero pivot in column 6
    _, _, stp = plan_result(Vz, s1, s2, seed)
    _, _, sts = static_call(Vz, s1, s2, seed)
    assert stp == (rc.E_RANK, 6) and sts == stp


def test_static_rejects_shapes_beyond_the_scratch():
    # 128 columns with s1 = 32768 need more workspace than the static array holds: refused on
    # the host before anything is launched
    m, n, s1, s2 = 100_000, 128, 32_768, 512
    assert rc.workspace_bytes(m, n, s1, s2) > rc.STATIC_WORKSPACE_BYTES
    V = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    Q = torch.empty_like(V)
    R = torch.empty((n, n), dtype=torch.float64, device="cuda")
    st = rc.lib().rcqr_factor_static(m, n, s1, s2, 1, 0, ctypes.c_void_p(V.data_ptr()), n, ctypes.c_void_p(Q.data_ptr()), n,
                                     ctypes.c_void_p(R.data_ptr()), n, None, None)
    assert st == rc.E_SCRATCH
    with pytest.raises(rc.RcqrError) as e:
        rc.factor_static(V, Q, R, s1, s2, 1)
    assert e.value.status == rc.E_SCRATCH
