"""The no-allocation pair call (twed_pair_noalloc) against twed_pair (GPU only).

twed_pair_noalloc runs the kernels of twed_pair with the library's fixed
per-device scratch array as workspace, so every result must equal the
twed_pair result bit for bit; the oracle bar of the single-pair tests (FP64
within 1e-12 relative, FP32 within 1e-5 of the FP64 oracle on the same
rounded inputs) is checked as well.  Two calls in a row, the second smaller,
catch state left in the shared array by the first (flags, ticket, offset).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2007_16135_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2007_16135_amd import binding as B  # noqa: E402

RTOL = {"f64": 1e-12, "f32": 1e-5, "f32_acc64": 1e-6, "auto": 1e-5}
LIMIT = 64 << 20


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def operands(A, TA, B_, TB, precision):
    dt = torch.float64 if precision == "f64" else torch.float32
    d = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    return d(A), d(TA), d(B_), d(TB)


def call_both(L, ops, nA, nB, prm, out_dt):
    """(twed_pair_noalloc value, twed_pair value), each through the C ABI."""
    A, TA, Bd, TB = ops
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out_n = torch.full((1,), float("nan"), dtype=out_dt, device="cuda")
    st = L.twed_pair_noalloc(A.data_ptr(), TA.data_ptr(), nA, Bd.data_ptr(), TB.data_ptr(), nB,
                             ctypes.byref(prm), out_n.data_ptr(), stream)
    assert st == 0, L.twed_last_error().decode()
    need = L.twed_pair_workspace_size(nA, nB, ctypes.byref(prm))
    assert 0 < need <= LIMIT
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out_w = torch.full((1,), float("nan"), dtype=out_dt, device="cuda")
    st = L.twed_pair(A.data_ptr(), TA.data_ptr(), nA, Bd.data_ptr(), TB.data_ptr(), nB,
                     ctypes.byref(prm), out_w.data_ptr(), ws.data_ptr(), ws.numel(), stream)
    assert st == 0, L.twed_last_error().decode()
    torch.cuda.synchronize()
    return out_n.item(), out_w.item()


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_acc64", "auto"])
def test_noalloc_equals_pair_two_calls(precision):
    L = B.load_library()
    out_dt = torch.float32 if precision == "f32" else torch.float64
    # the first call is larger (many strips, several workgroups), the second smaller
    for nA, nB, dim, p, seed in ((6000, 5000, 3, 2.0, 1), (700, 450, 3, 2.0, 2), (90, 130, 1, 1.0, 3)):
        c = synth.random_pair(seed, seed + 10, nA, nB, dim, irregular=True, nu=0.01, lam=0.5, p=p)
        A, TA, Bs, TB = c.A, c.TA, c.B, c.TB
        if precision != "f64":
            A, TA, Bs, TB = (np.asarray(x, dtype=np.float32) for x in (A, TA, Bs, TB))
        prm = B.make_params(0.01, 0.5, p, dim, precision)
        say(f"noalloc {precision}: {nA} x {nB}, dim {dim}")
        got, want = call_both(L, operands(A, TA, Bs, TB, precision), nA, nB, prm, out_dt)
        assert got == want, (got, want)
        f64 = lambda x: np.asarray(x, dtype=np.float64)
        ref = oracle.get().twed(f64(A).reshape(nA, -1), f64(TA), f64(Bs).reshape(nB, -1), f64(TB),
                                0.01, 0.5, p, rows=True)
        assert abs(got - ref) <= RTOL[precision] * ref, (got, ref)


def test_noalloc_near_the_limit():
    # a pair whose workspace is just under the array size, then a small one;
    # both bitwise equal to twed_pair
    L = B.load_library()
    prm = B.make_params(1e-3, 1.0, 1.0, 1, "f32")
    nB = 3000
    lo, hi = 1, 1 << 24
    while lo < hi:
        m = (lo + hi + 1) // 2
        if L.twed_pair_workspace_size(m, nB, ctypes.byref(prm)) <= LIMIT:
            lo = m
        else:
            hi = m - 1
    nA = lo
    assert L.twed_pair_workspace_size(nA + 1, nB, ctypes.byref(prm)) > LIMIT
    rng = np.random.default_rng(9)
    for n_a in (nA, 257):
        A = synth.walk(rng, n_a, 1).astype(np.float32)
        Bs = synth.walk(rng, nB, 1).astype(np.float32)
        TA = np.arange(n_a, dtype=np.float32)
        TB = np.arange(nB, dtype=np.float32)
        say(f"noalloc near the limit: {n_a} x {nB}")
        got, want = call_both(L, operands(A, TA, Bs, TB, "f32"), n_a, nB, prm, torch.float32)
        assert got == want, (n_a, got, want)
        assert np.isfinite(got)
