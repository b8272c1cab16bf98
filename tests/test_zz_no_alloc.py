"""tclbm_moments_noalloc (the moments entry point for callers that cannot
allocate) against tclbm_moments, through the C ABI: the same fields and the
same FP64 sums, bitwise, on two calls in a row, the second on a smaller
lattice (so that it meets the first call's leftovers in the shared device
array), with and without fields."""
import sys

import numpy as np
import pytest

from paper_1610_07114_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_07114_amd import tclbm
    return tclbm


def _same(T, case, storage, steps):
    lat = T.Lattice(case, storage=storage)
    lat.step(steps)
    nx, ny = case.nx, case.ny
    ref = T.tclbm_moments(lat.h, nx, ny, fields=True)
    got = T.tclbm_moments_noalloc(lat.h, nx, ny, fields=True)
    sums_only = T.tclbm_moments_noalloc(lat.h, nx, ny, fields=False)
    lat.close()
    for a, b in zip(ref[:4], got[:4]):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
    assert ref[5] == got[5] == sums_only[5] == T.OK
    assert ref[4].as_dict() == got[4].as_dict() == sums_only[4].as_dict()
    return ref[4].as_dict()


def test_noalloc_moments_equal_moments_on_two_calls(T):
    # 700 x 400 = 280,000 nodes: 1094 blocks of 256, three chunks, the last
    # block partly filled
    big = W.rayleigh_benard(nx=700, ny=400, seed=2, noise=1e-3)
    say("case moments without allocation: 700x400 rayleigh-benard fp32, 30 steps")
    s = _same(T, big, "f32", 30)
    say(f"  sums {s}")
    small = W.uniform_noise(64, 40, seed=3, ax=1e-5)
    say("case moments without allocation: 64x40 periodic fp16, 20 steps (after the larger call)")
    s = _same(T, small, "f16", 20)
    say(f"  sums {s}")
