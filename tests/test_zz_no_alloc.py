"""fcns_fc_derivative_noalloc (no context, tables in the library's static
device array) against fcns_fc_derivative on the same lines, through the C
ABI: two calls in a row, the second with a smaller input (another N', another
order), each within the FP64 bar of 1e-11 relative L2 of the context's
result and of the oracle; sizes beyond the array are refused."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle.fcgram import fc_derivative_lines

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fcns():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2002_01392_amd as P
    P.load_library()
    return P


def rel_l2(a, b):
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    b = b.detach().cpu().numpy() if hasattr(b, "detach") else np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _lines(nz, lz, n, seed):
    z = np.linspace(0, lz, nz)
    r = W.rng(seed)
    return np.stack([np.sin(r.uniform(1, 9) * z + r.uniform()) * np.exp(r.uniform(-1, 1) * z)
                     for _ in range(n)])


def _noalloc(fcns, nz, lz, d, C, order, f):
    from paper_2002_01392_amd import fctable
    lib = fcns.load_library()
    tab = np.ascontiguousarray(fctable.load(d, C), dtype=np.float64)
    fin = torch.from_numpy(f).to("cuda").contiguous()
    out = torch.empty_like(fin)
    stream = torch.cuda.current_stream()
    st = lib.fcns_fc_derivative_noalloc(nz, lz, d, C, tab.ctypes.data_as(ctypes.c_void_p),
                                        order, ctypes.c_void_p(fin.data_ptr()), f.shape[0], 1,
                                        nz, ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    return out


def test_noalloc_fc_derivative_matches_the_context_call(fcns):
    cases = [(257, 1.7, 5, 31, 1, 513), (65, 1.0, 5, 25, 2, 77)]   # second call smaller
    for nz, lz, d, C, order, n in cases:
        f = _lines(nz, lz, n, 900 + nz)
        got = _noalloc(fcns, nz, lz, d, C, order, f)
        s = fcns.Solver(8, 8, nz, 1.0, 1.0, lz, 0.0, d=d, C=C)
        ref = s.fc_derivative(torch.from_numpy(f), order)
        torch.cuda.synchronize()
        assert rel_l2(got, ref) < 1e-11, (nz, C, order)
        assert rel_l2(got, fc_derivative_lines(f, d, C, lz, order)) < 1e-11, (nz, C, order)
        s.close()


def test_noalloc_refuses_sizes_beyond_its_array(fcns):
    lib = fcns.load_library()
    dummy = np.zeros(4096)
    buf = torch.zeros(8, device="cuda", dtype=torch.float64)
    p = ctypes.c_void_p(buf.data_ptr())
    tp = dummy.ctypes.data_as(ctypes.c_void_p)
    # N' = 513 + 25 > 512
    assert lib.fcns_fc_derivative_noalloc(513, 1.0, 5, 25, tp, 1, p, 1, 1, 513, p, None) == -1
    # C d = 37 * 7 > 256
    assert lib.fcns_fc_derivative_noalloc(65, 1.0, 7, 37, tp, 1, p, 1, 1, 65, p, None) == -1
    # odd N', bad order
    assert lib.fcns_fc_derivative_noalloc(64, 1.0, 5, 25, tp, 1, p, 1, 1, 64, p, None) == -1
    assert lib.fcns_fc_derivative_noalloc(65, 1.0, 5, 25, tp, 3, p, 1, 1, 65, p, None) == -1
    # zero lines: nothing to do
    assert lib.fcns_fc_derivative_noalloc(65, 1.0, 5, 25, tp, 1, p, 0, 1, 65, p, None) == 0
