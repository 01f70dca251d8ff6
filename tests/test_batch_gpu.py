"""GPU tests of the batched form (include/gs_batch.h): every problem of a
batch against the same problem advanced alone through gs_fluid (bit-identical
with the same launch shape: each work item is exactly one workgroup of the
single-problem kernel) and against the CPU oracle; graph replays against
direct launches; time clipping; the autotuner and its cache."""
import sys

import numpy as np
import pytest

import workloads as wl
from tests.parity import oracle_run, rel_linf, to_cpu, to_gpu

pytestmark = pytest.mark.gpu

DIMS = [(24, 16, 12), (40, 24, 20), (16, 32, 8), (33, 17, 9), (20, 20, 20), (48, 8, 16)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problems(dims, seed0=200):
    out = []
    for i, (nx, ny, nz) in enumerate(dims):
        v = (0.4, -0.3, 0.2) if i % 2 else (0.0, 0.0, 0.0)
        out.append(wl.random_plane(nx, ny, nz, seed=seed0 + i, v=v))
    return out


def _state(U0, dtype, bc):
    from paper_1812_07977_amd import Fluid
    nz, ny, nx = U0.shape[1:]
    with Fluid((nx, ny, nz), bc=bc, dtype=dtype) as F:
        return F.state_from(U0)


def _alone(U0, dtype, bc, nsteps, launch, t_end=0.0):
    from paper_1812_07977_amd import Fluid
    nz, ny, nx = U0.shape[1:]
    with Fluid((nx, ny, nz), bc=bc, dtype=dtype) as F:
        F.set_launch(*launch)
        S = F.state_from(U0)
        F.advance(S, nsteps, t_end)
        t = F.time
        return to_cpu(S), t


@pytest.mark.parametrize("dtype,bc", [("f64", "outflow"), ("f64", "periodic"),
                                      ("f32", "periodic"), ("f32", "outflow")])
def test_batch_equals_each_problem_alone(dtype, bc):
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS)
    launch = (16, 8) if dtype == "f64" else (8, 8)
    _say(f"case: batch of {len(DIMS)} {dtype} {bc}, 6 steps, launch {launch}")
    states = [_state(U0, dtype, bc) for U0 in probs]
    with Batch(DIMS, states, bc=bc, dtype=dtype) as B:
        B.set_launch(*launch)
        B.advance(6)
        times = B.times()
        got = [to_cpu(S) for S in states]
    for i, U0 in enumerate(probs):
        ref, t = _alone(U0, dtype, bc, 6, launch)
        assert np.array_equal(got[i], ref), i
        assert times[i] == t, i


def test_batch_matches_the_oracle():
    from paper_1812_07977_amd.batch import Batch
    dims = [(24, 16, 12), (33, 17, 9), (20, 28, 14)]
    probs = _problems(dims, seed0=300)
    n = 8
    states = [to_gpu(U0) for U0 in probs]
    with Batch(dims, states, bc="outflow") as B:
        B.advance(n)
        times = B.times()
        got = [to_cpu(S) for S in states]
    for i, U0 in enumerate(probs):
        ref, dts = oracle_run(U0, "outflow", n)
        assert max(rel_linf(got[i], ref)) <= 1e-12, i
        assert abs(times[i] - float(np.sum(dts))) <= 1e-14 * n * float(np.sum(dts)), i


def test_graph_replays_match_direct_launches():
    import torch
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS, seed0=400)
    sa = [to_gpu(U0) for U0 in probs]
    sb = [to_gpu(U0) for U0 in probs]
    with Batch(DIMS, sa, bc="periodic") as A, Batch(DIMS, sb, bc="periodic") as Bd:
        for call in range(4):
            A.advance(3, graph=True)
            Bd.advance(3, graph=False)
            A.sync()
            Bd.sync()
            # unrelated eager work between replays
            x = torch.randn(1 << 20, device="cuda")
            torch.cuda.synchronize()
            del x
            for i in range(len(DIMS)):
                assert torch.equal(sa[i], sb[i]), (call, i)
            assert A.times() == Bd.times()


def test_time_clipping_per_problem():
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS[:4], seed0=500)
    states = [to_gpu(U0) for U0 in probs]
    with Batch(DIMS[:4], states, bc="outflow") as B:
        B.advance(200, t_end=0.02)
        times = B.times()
        before = [to_cpu(S) for S in states]
        B.advance(5, t_end=0.02)         # everything is at t_end: nothing moves
        after = [to_cpu(S) for S in states]
    assert all(t == 0.02 for t in times), times
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


def test_zero_steps_change_nothing():
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS[:3], seed0=550)
    states = [to_gpu(U0) for U0 in probs]
    with Batch(DIMS[:3], states, bc="periodic") as B:
        B.advance(0)
        B.sync()
        assert B.times() == [0.0, 0.0, 0.0]
        for S, U0 in zip(states, probs):
            assert np.array_equal(to_cpu(S), U0)
        B.advance(2)
        ta = B.times()
        after = [to_cpu(S) for S in states]
    others = [to_gpu(U0) for U0 in probs]
    with Batch(DIMS[:3], others, bc="periodic") as C:
        C.advance(2)
        assert C.times() == ta
        for a, S in zip(after, others):
            assert np.array_equal(a, to_cpu(S))


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS, seed0=600)
    states = [to_gpu(U0) for U0 in probs]
    start = [to_cpu(S).copy() for S in states]
    cache = tmp_path / "tune.txt"
    with Batch(DIMS, states, bc="periodic") as B:
        ty, kz, hit = B.autotune(cache)
        assert (ty, kz, hit)[2] is False
        assert ty in (8, 16) and kz in (16, 32, 64)
        # tuning ran on scratch copies: states and times untouched
        for s0, S in zip(start, states):
            assert np.array_equal(s0, to_cpu(S))
        assert B.times() == [0.0] * len(DIMS)
    assert cache.read_text().strip()
    with Batch(DIMS, states, bc="periodic") as B:
        assert B.autotune(cache) == (ty, kz, True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_steps_after_autotune_match_problems_alone(dtype):
    # the autotuner launches every candidate shape (different grids and item
    # counts) through the same work-item counters; the steps after it, direct
    # and replayed, must still cover every item of every problem
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS, seed0=650)
    states = [_state(U0, dtype, "periodic") for U0 in probs]
    _say(f"case: batch {dtype} periodic, autotune then 4 direct + 3 replayed steps")
    with Batch(DIMS, states, bc="periodic", dtype=dtype) as B:
        ty, kz, _ = B.autotune()
        B.advance(4, graph=False)
        B.advance(3, graph=True)
        times = B.times()
        got = [to_cpu(S) for S in states]
    for i, U0 in enumerate(probs):
        ref, t = _alone(U0, dtype, "periodic", 7, (ty, kz))
        assert np.array_equal(got[i], ref), i
        assert times[i] == t, i


def test_nonphysical_problem_is_reported():
    from paper_1812_07977_amd import NonPhysicalError
    from paper_1812_07977_amd.batch import Batch
    probs = _problems(DIMS[:3], seed0=700)
    probs[1][0, 2, 3, 4] = -1.0
    states = [to_gpu(U0) for U0 in probs]
    with Batch(DIMS[:3], states, bc="outflow") as B:
        B.advance(1)
        with pytest.raises(NonPhysicalError):
            B.times()
        B.times()   # reported once


# ---------------------------------------------------------------------------
# the stated batch: 64 seeded Riemann problems, meshes drawn from 32..160
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_batch_of_64_matches_problems_alone(dtype):
    from paper_1812_07977_amd.batch import Batch
    dims, probs = wl.random_batch(64, seed=1)
    _say(f"case: batch of 64 (32..160) {dtype} periodic, autotuned, 2 steps")
    states = [_state(U0, dtype, "periodic") for U0 in probs]
    with Batch(dims, states, bc="periodic", dtype=dtype) as B:
        ty, kz, _ = B.autotune()
        B.advance(2)
        times = B.times()
        sample = [0, 17, 40, 63]
        got = {i: to_cpu(states[i]) for i in sample}
    for i in sample:
        ref, t = _alone(probs[i], dtype, "periodic", 2, (ty, kz))
        assert np.array_equal(got[i], ref), i
        assert times[i] == t, i
    if dtype == "f64":
        # the benchmark's batch in its timed configuration, against the oracle
        for i in sample:
            ref, dts = oracle_run(probs[i], "periodic", 2)
            assert max(rel_linf(got[i], ref)) <= 1e-12, i
            assert abs(times[i] - float(np.sum(dts))) <= 1e-14 * 2 * float(np.sum(dts)), i


@pytest.mark.parametrize("dtype,bc", [("f64", "outflow"), ("f64", "periodic"), ("f32", "outflow")])
def test_degenerate_meshes_in_a_batch(dtype, bc):
    # one-cell-thick and tiny meshes beside a ragged one: every work item
    # maps its ghost columns and planes to valid cells
    from paper_1812_07977_amd.batch import Batch
    dims = [(1, 1, 7), (2, 2, 2), (64, 1, 1), (5, 33, 17), (1, 9, 1)]
    probs = _problems(dims, seed0=800)
    _say(f"case: degenerate batch {dims} {dtype} {bc}, 4 steps")
    states = [_state(U0, dtype, bc) for U0 in probs]
    with Batch(dims, states, bc=bc, dtype=dtype) as B:
        B.advance(4)
        times = B.times()
        got = [to_cpu(S) for S in states]
    for i, U0 in enumerate(probs):
        ref, t = _alone(U0, dtype, bc, 4, (0, 0))
        assert np.array_equal(got[i], ref), i
        assert times[i] == t, i


def test_batch_of_one_matches_the_oracle():
    from paper_1812_07977_amd.batch import Batch
    dims = [(40, 24, 20)]
    probs = _problems(dims, seed0=900)
    _say("case: batch of one 40x24x20 outflow, 10 steps")
    states = [to_gpu(probs[0])]
    with Batch(dims, states, bc="outflow") as B:
        B.advance(10)
        times = B.times()
        got = to_cpu(states[0])
    ref, dts = oracle_run(probs[0], "outflow", 10)
    assert max(rel_linf(got, ref)) <= 1e-12
    assert abs(times[0] - float(np.sum(dts))) <= 1e-14 * 10 * float(np.sum(dts))


def test_the_largest_count_of_small_problems():
    # 65536 problems, the most a batch takes, each 1..4 cells per side
    # (one-cell and two-cell dimensions included), periodic, against the
    # oracle problem by problem: the instance table, its binary search and
    # the XCD shares of the work items at their largest
    from paper_1812_07977_amd.batch import Batch
    count, n = 1 << 16, 2
    rng = np.random.default_rng(4242)
    dims = [tuple(int(v) for v in rng.integers(1, 5, 3)) for _ in range(count)]
    probs = [wl.random_plane(nx, ny, nz, seed=10000 + i, v=(0.2, -0.1, 0.3))
             for i, (nx, ny, nz) in enumerate(dims)]
    _say(f"case: batch of {count} problems of 1..4 cells per side, periodic, {n} steps")
    states = [to_gpu(U0) for U0 in probs]
    with Batch(dims, states, bc="periodic") as B:
        B.advance(n)
        times = B.times()
        got = [to_cpu(S) for S in states]
    worst = 0.0
    for i, U0 in enumerate(probs):
        ref, dts = oracle_run(U0, "periodic", n)
        e = max(rel_linf(got[i], ref))
        worst = max(worst, e)
        assert e <= 1e-12, (i, dims[i], e)
        assert abs(times[i] - float(np.sum(dts))) <= 1e-14 * n * float(np.sum(dts)), i
    _say(f"largest relative L-infinity difference {worst:.2e}")
