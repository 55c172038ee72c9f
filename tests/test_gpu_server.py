"""The serving loop (fa_server_*): continuous admission by workspace memory,
concurrent solves on several streams, and results identical (bitwise) to the
same solves run alone.  Exactness against the oracle is the business of
test_gpu_parity.py; here the reference is the library's own solo solve."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06684_amd as fa
    fa.lib()


def fa():
    import paper_2401_06684_amd as m
    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _ops():
    m = fa()
    cd = m.Stencil7((24, 20, 18), wl.convdiff_stencil(24, 50.0))
    cd.poly_setup(8, "cheb")
    lap = m.Stencil7((64, 64, 1), wl.laplace_stencil(2), hermitian=True)
    lap.poly_setup(4, "cheb")
    rp, ci, va = wl.stencil_csr((16, 16, 1), wl.laplace_stencil(2))
    csr = m.CSR(rp, ci, va, hermitian=True)
    csr.set_spectral_interval(*_interval2d(16))
    csr.poly_setup(0)
    U = wl.su3_links(4, eps=0.3, seed=1)
    wil = m.Wilson(U, 0.05)
    wil.poly_setup(4, "ritz", start=dev(wl.rhs(wil.n, seed=11, complex_=True)))
    return [cd, lap, csr, wil]


def _interval2d(N):
    import math
    c = math.cos(math.pi / (N + 1))
    return 4 - 4 * c, 4 + 4 * c


def _requests(ops, count):
    reqs = []
    for i in range(count):
        op = ops[i % len(ops)]
        cplx = op.dtype == torch.complex128
        b = dev(wl.rhs(op.n, seed=100 + i, complex_=cplx))
        kind = "sqrt" if i % 3 == 1 else "invsqrt"
        tol = 1e-6 if i % 2 else 1e-10
        reqs.append((op, b, kind, tol))
    return reqs


def test_results_in_the_mix_equal_solo_results():
    ops = _ops()
    reqs = _requests(ops, 24)
    solo = []
    for op, b, kind, tol in reqs:
        x, st = op.apply(b, kind=kind, m_max=120, tol=tol)
        assert st["converged"], (op, kind, tol)
        solo.append(x.clone())
    torch.cuda.synchronize()
    srv = fa().Server(1 << 30, n_workers=4)
    tickets = [srv.submit(op, b, kind=kind, m_max=120, tol=tol) for op, b, kind, tol in reqs]
    for t, ref in zip(tickets, solo):
        x, info = srv.wait(t)
        assert info["status"] == 0
        assert torch.equal(x, ref)
    s = srv.status()
    assert s["completed"] == len(reqs) and s["pending"] == 0 and s["inflight"] == 0
    assert s["peak_inflight"] >= 2          # solves overlapped
    assert s["bytes_inflight"] == 0 and s["largest_free"] == s["pool_bytes"]
    srv.close()


def test_admission_by_workspace_memory():
    m = fa()
    op = m.Stencil7((32, 32, 32), wl.convdiff_stencil(32, 50.0))
    op.poly_setup(8, "cheb")
    need = op.workspace_bytes(60)
    srv = m.Server(2 * need + 1024, n_workers=4)   # room for two solves at a time
    b = dev(wl.rhs(op.n, seed=0))
    ref, _ = op.apply(b, m_max=60, tol=1e-10)
    tickets = [srv.submit(op, b, m_max=60, tol=1e-10) for _ in range(8)]
    for t in tickets:
        x, info = srv.wait(t)
        assert torch.equal(x, ref)
        assert info["ws_bytes"] == need
        assert info["t_submit_ms"] <= info["t_start_ms"] <= info["t_done_ms"]
    s = srv.status()
    assert s["peak_inflight"] <= 2 and s["peak_bytes_inflight"] <= 2 * need + 1024
    # a request that can never fit is refused at submit
    with pytest.raises(m.FAError) as e:
        srv.submit(op, b, m_max=200, tol=1e-10)
    assert e.value.status == m._lib.FA_ERR_WORKSPACE
    srv.close()


def test_failed_request_does_not_stop_the_server():
    m = fa()
    ops = _ops()
    wil = ops[3]
    srv = m.Server(1 << 28, n_workers=2)
    b = dev(wl.rhs(wil.n, seed=3, complex_=True))
    bad = srv.submit(wil, b, m_max=50, tol=1e-8, mixed=True)   # FP32 chain: stencil + Chebyshev only
    good = srv.submit(wil, b, m_max=200, tol=1e-8)
    with pytest.raises(m.FAError) as e:
        srv.wait(bad)
    assert e.value.status == m._lib.FA_ERR_UNSUPPORTED
    x, info = srv.wait(good)
    assert info["status"] == 0 and info["stats"]["converged"] == 1
    ref, _ = wil.apply(b, m_max=200, tol=1e-8)
    assert torch.equal(x, ref)
    srv.close()
