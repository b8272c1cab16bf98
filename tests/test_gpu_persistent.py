"""Persistent batched launches (tclbm_batch_set_persistent): many steps of
every member per cooperative launch, with a bounded grid barrier between
steps.  The states must be bitwise those of the same lattices stepped alone,
in FP32 and in 16-bit storage (whose rounding generator advances per step
inside the launch), and a barrier whose wait runs out must be reported, not
hang.  The failure case is forced from the host with a 1 us wait limit: the
first block to reach the barrier gives up at once, and every wave still ends
normally."""
import numpy as np
import pytest

from paper_1610_07114_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_1610_07114_amd import tclbm
    return tclbm


def say(msg):
    print(msg, flush=True)


def default_cases():
    # every member on the default scheme (walls, bounce-back ends, periodic)
    return [W.rayleigh_benard(nx=130, ny=67, seed=1, noise=1e-3), W.couette(),
            W.shock_tube(nx=700, ny=5), W.uniform_noise(64, 40, seed=2, ax=1e-5),
            W.rayleigh_benard(nx=300, ny=150, seed=4, noise=1e-3)]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_persistent_batch_equals_members_alone_bitwise(T, storage):
    import torch
    cases = default_cases()
    say(f"case persistent batch of {len(cases)} uneven lattices {storage}, 75 steps, vs alone")
    stream = torch.cuda.Stream()
    alone = []
    for cs in cases:
        a = T.Lattice(cs, storage=storage, stream=stream)
        a.step(75)
        alone.append(a.read_state())
        a.close()
    lats = [T.Lattice(cs, storage=storage, stream=stream) for cs in cases]
    b = T.Batch(lats)
    b.set_persistent(8)
    assert b.persistent == 8
    assert b.kernel.startswith("batch_persistent_kernel")
    b.step(33)                   # four launches of 8 steps and one of 1
    b.set_strip_rows(5)          # launch shape changed mid-run
    b.step(21)
    b.set_persistent(64)
    b.step(16)                   # one launch shorter than the limit
    b.set_persistent(0)          # back to per-step launches
    assert b.kernel.startswith("batch_step_kernel")
    b.step(5)
    b.close()
    for lat, ref in zip(lats, alone):
        assert lat.steps == 75
        assert np.array_equal(lat.read_state(), ref)
        lat.close()


def test_persistent_batch_timed_matches_graph_path(T):
    """tclbm_batch_step_timed through persistent launches: a successful
    launch reports OK and leaves the state of the per-step graph path."""
    import torch
    cases = [W.rayleigh_benard(nx=256, ny=128, seed=s, noise=1e-3) for s in range(3)]
    say("case persistent vs graph-replayed batch, 3 x 256x128 fp32, 40 steps")
    stream = torch.cuda.Stream()
    states = []
    for persist in (0, 10):
        lats = [T.Lattice(cs, storage="f32", stream=stream) for cs in cases]
        b = T.Batch(lats)
        b.set_graph_chunk(8)
        b.set_persistent(persist)
        ms = b.step_timed(40)
        assert ms > 0
        b.close()
        states.append([lat.read_state() for lat in lats])
        for lat in lats:
            lat.close()
    for x, y in zip(*states):
        assert np.array_equal(x, y)


def test_persistent_needs_default_scheme_and_32_or_16_bit(T):
    import torch
    stream = torch.cuda.Stream()
    say("case persistent refused: generic-scheme member, FP64 storage")
    lats = [T.Lattice(cs, storage="f32", stream=stream)
            for cs in (W.couette(), W.couette_variable_viscosity(Pr=4.0, gamma=1.5))]
    b = T.Batch(lats)
    with pytest.raises(T.TclbmError) as ei:
        b.set_persistent(8)
    assert ei.value.status == T.E_INVALID
    assert b.persistent == 0
    b.step(4)
    b.close()
    for lat in lats:
        lat.close()
    lat = T.Lattice(W.couette(), storage="f64", stream=stream)
    b = T.Batch([lat])
    with pytest.raises(T.TclbmError) as ei:
        b.set_persistent(8)
    assert ei.value.status == T.E_INVALID
    with pytest.raises(T.TclbmError) as ei:
        b.set_persistent(-1)
    assert ei.value.status == T.E_INVALID
    b.close()
    lat.close()


def test_persistent_barrier_wait_limit_is_reported(T):
    """With a 1 us limit the blocks that reach a barrier first give up:
    the launch ends, step_timed reports E_DEVICE, the members are marked
    unstable and the batch refuses further steps."""
    import torch
    stream = torch.cuda.Stream()
    cases = [W.rayleigh_benard(nx=256, ny=128, seed=s, noise=1e-3) for s in range(6)]
    say("case persistent barrier wait limit 1 us, 6 x 256x128 fp32 (bounded; every wave exits)")
    lats = [T.Lattice(cs, storage="f32", stream=stream) for cs in cases]
    b = T.Batch(lats)
    b.set_persistent(16, wait_us=1)
    with pytest.raises(T.TclbmError) as ei:
        b.step_timed(16)
    assert ei.value.status == T.E_DEVICE
    with pytest.raises(T.TclbmError) as ei:
        b.step(1)
    assert ei.value.status == T.E_STATE
    b.close()
    for lat in lats:
        with pytest.raises(T.TclbmError) as ei:
            lat.step(1)
        assert ei.value.status == T.E_STATE
        lat.close()
