"""hbt_perm_test_static (the entry point that allocates nothing) against
hbt_perm_test with a caller workspace: two calls in a row on the library's
device scratch, the second with a smaller input, both equal to the workspace
call and to the oracle's counts; a test too large for the scratch is refused
before anything runs."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_08048_amd import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_2605_08048_amd import hbt  # noqa: E402

DEV = "cuda:0"


def _pair(n, m, d, seed):
    g = np.random.default_rng([21, seed])
    mu = synth.random_unit(g, d)
    mv = synth.direction_at_angle(g, mu, 35.0)
    X = synth.unit_rows(2.2 * mu + g.standard_normal((n, d)) / math.sqrt(d)).astype(np.float32)
    Y = synth.unit_rows(2.2 * mv + g.standard_normal((m, d)) / math.sqrt(d)).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("prec", ["bf16x2", "f32", "i8x3", "bf16lazy"])
def test_static_scratch_matches_workspace_call(prec):
    # the second call is smaller: it must not see anything the first left behind
    for n, m, d, B in [(3000, 2000, 1024, 6000), (300, 170, 96, 900)]:
        print(f"static scratch {prec}: n={n} m={m} d={d} B={B}", flush=True)
        X, Y = _pair(n, m, d, seed=n + d)
        Xd, Yd = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
        a = hbt.perm_test(Xd, Yd, B, seed=5, precision=prec, want_T="f64", want_masks=True)
        b = hbt.perm_test(Xd, Yd, B, seed=5, precision=prec, want_T="f64", want_masks=True,
                          static_scratch=True)
        for k in ["count", "n_recheck", "status", "B", "h_identity", "t_obs", "p", "r_x", "r_y", "t_mean", "t_sd"]:
            assert a[k] == b[k], (prec, n, k, a[k], b[k])
        assert np.array_equal(a["masks"], b["masks"])
        assert np.array_equal(a["T"], b["T"])
        o = O.perm_test(X, Y, B, seed=5, want_T=True)
        tie = int(np.sum(np.abs(o["T"] - o["t_obs"]) <= 1e-6 * abs(o["t_obs"])))
        assert abs(b["count"] - o["count"]) <= tie and b["status"] == 0


def test_static_scratch_refuses_tests_larger_than_it():
    L = hbt.lib()
    prm = hbt.make_params(8000, 8000, 1024, 20000, precision="bf16x2")
    assert L.hbt_perm_test_workspace_size(C.byref(prm)) > 64 << 20
    X = torch.zeros(8000 * 1024, dtype=torch.float32, device=DEV)
    res = torch.zeros(hbt.RESULT_BYTES, dtype=torch.uint8, device=DEV)
    st = L.hbt_perm_test_static(C.c_void_p(X.data_ptr()), C.c_void_p(X.data_ptr()), C.byref(prm),
                                C.c_void_p(res.data_ptr()), None, None, None)
    assert st == hbt.ERR_WORKSPACE
    assert b"static scratch" in L.hbt_last_error()
    assert int(res.sum()) == 0  # nothing ran
