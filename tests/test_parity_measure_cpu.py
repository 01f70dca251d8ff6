"""The per-field error measures of the GPU parity tests, on the CPU: a
field that is zero in exact arithmetic, whether the reference holds exact
zeros or rounding-level values, is measured against the largest field."""
import numpy as np

from tests.parity import ZERO_FIELD, rel_l1, rel_linf


def _ref():
    ref = np.zeros((5, 2, 3, 4))
    ref[0] = 1.0
    ref[1] = 7.9
    ref[4] = 34.0
    ref[2, 0, 0, 0] = 7e-16      # rounding-level transverse momentum
    return ref


def test_rounding_level_field_is_scaled_by_the_largest_field():
    ref = _ref()
    gpu = ref.copy()
    gpu[2] += 1e-8
    gpu[3] += 1e-8               # exactly zero in the reference
    linf = rel_linf(gpu, ref)
    assert np.isclose(linf[2], 1e-8 / 34.0) and np.isclose(linf[3], 1e-8 / 34.0)
    l1 = rel_l1(gpu, ref)
    big = 34.0 * 24
    assert np.isclose(l1[2], 24e-8 / big) and np.isclose(l1[3], 24e-8 / big)


def test_ordinary_fields_keep_their_own_scale():
    ref = _ref()
    ref[2] = 2e-9 * 34.0         # small but above the zero-field threshold
    assert 2e-9 > ZERO_FIELD
    gpu = ref.copy()
    gpu[0] += 1e-6
    gpu[2] += 1e-12
    linf = rel_linf(gpu, ref)
    assert np.isclose(linf[0], 1e-6) and np.isclose(linf[2], 1e-12 / (2e-9 * 34.0))
    assert rel_linf(ref, ref) == [0.0] * 5
