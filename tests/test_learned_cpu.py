"""Host logic of the learned-correction driver (paper_1812_07977_amd/learned.py)
that needs no GPU: advancing the fine reference to a coarse step's end time."""
import pytest

from paper_1812_07977_amd import learned


class _FakeFine:
    """Stands in for a Fluid with device dt: each step advances the time by
    dt, clipped to t_end, as gs_fluid_advance does."""

    def __init__(self, dt):
        self.dt, self.time, self.steps = dt, 0.0, 0

    def advance(self, U, nsteps, t_end):
        for _ in range(nsteps):
            self.steps += 1
            if not self.time < t_end:
                continue
            self.time = min(self.time + self.dt, t_end)


def test_advance_to_stops_once_the_end_time_is_reached():
    F = _FakeFine(dt=0.3)
    learned._advance_to(F, None, 1.0)
    assert F.time == 1.0
    assert F.steps == 4           # two chunks of two: 0.3, 0.6, 0.9, 1.0


def test_advance_to_raises_if_the_end_time_is_never_reached():
    F = _FakeFine(dt=0.0)         # a solve that does not move
    with pytest.raises(RuntimeError):
        learned._advance_to(F, None, 1.0, limit=5)
    assert F.steps == 10


@pytest.mark.parametrize("mode", [0, 1])
def test_input_features_match_the_oracle(mode):
    # the statistics of the network's inputs are taken on features that the
    # driver computes in torch; they must be the features the kernels feed
    # the network (mode 1 is checked against the same oracle function on the
    # GPU), here against the oracle on a seeded state with large velocities
    import numpy as np
    import torch

    import oracle.cnn as ocnn
    import workloads as wl
    U = wl.random_plane(12, 10, 8, seed=4, v=(1.5, -0.7, 0.3))
    got = learned.input_features(torch.from_numpy(U), mode).numpy()
    want = U if mode == 0 else ocnn.features(U, 1.4)
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=1e-14, atol=1e-14)
