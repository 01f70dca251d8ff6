"""GPU tests of the learned-correction kernels against the CPU oracle
(oracle/cnn.py), through the C ABI (include/gs_cnn.h).

The GPU multiplies BF16 operands and accumulates in FP32.  The oracle is
handed exactly the operands the GPU sees (weights and activations rounded to
BF16 between layers, oracle.cnn.bf16_round) and computes in FP64:
  - with dyadic weights and inputs chosen so that every product and partial
    sum is exact in FP32, the two sides must agree bit for bit, whatever the
    summation order (forward pass);
  - with ordinary random values, FP32 and FP64 sums differ by at most about
    K u sum |terms| (K terms, u = 2^-24), and where that straddles a BF16
    rounding boundary of a hidden activation the two sides round it one
    BF16 unit apart; the tests bound both effects from absolute values
    computed by the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu

HIDDEN_CH = 32


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _net(shape, bc="periodic"):
    from paper_1812_07977_amd.learned import CorrectionNet
    return CorrectionNet(shape, bc=bc)


def _pair(head):
    """An FP32 state pair with the given head and zero compensation."""
    import torch
    h = torch.from_numpy(np.ascontiguousarray(head, dtype=np.float32))
    return torch.stack([h, torch.zeros_like(h)]).contiguous().cuda()


def _oracle_forward_bf16(x, params, bc):
    """The network with the GPU's roundings: BF16 weights, BF16 activations
    after each ReLU, FP64 sums."""
    (w1, b1), (w2, b2), (w3, b3) = params
    r = ocnn.bf16_round
    a1 = ocnn.conv3(x, r(w1), b1, bc)
    h1 = r(ocnn.relu(a1))
    a2 = ocnn.conv3(h1, r(w2), b2, bc)
    h2 = r(ocnn.relu(a2))
    y = ocnn.conv3(h2, r(w3), b3, bc)
    return y, (a1, h1, a2, h2)


def _params_from_flat(flat):
    from paper_1812_07977_amd.learned import split_params
    p = [a.astype(np.float64) for a in split_params(flat)]
    return [(p[0], p[1]), (p[2], p[3]), (p[4], p[5])]


def _dyadic_params(rng):
    """Sparse weights in {0, +-1/8} (density 0.2 in the first layer, 0.1 after)
    and biases in multiples of 1/16, so every
    sum of the network is exact in FP32."""
    from paper_1812_07977_amd.learned import SHAPES
    parts = []
    for k, s in enumerate(SHAPES):
        if len(s) == 1:
            parts.append(rng.integers(-4, 5, s) / 16.0)
        else:
            dens = 0.2 if k == 0 else 0.1
            w = rng.choice([-0.125, 0.125], s) * (rng.random(s) < dens)
            parts.append(w)
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


@pytest.mark.parametrize("shape,bc", [((32, 16, 8), "periodic"), ((20, 12, 6), "outflow"),
                                      ((16, 16, 16), "periodic"),
                                      # 16 tiles and 160 planes: workgroups march 2 planes
                                      ((64, 64, 160), "periodic"),
                                      # degenerate meshes: one cell, one row, one plane;
                                      # every halo cell maps back into the mesh
                                      ((1, 1, 1), "periodic"), ((1, 1, 1), "outflow"),
                                      ((17, 1, 3), "outflow"), ((3, 2, 1), "periodic"),
                                      ((1, 40, 2), "periodic")])
def test_forward_is_bit_exact_on_exactly_representable_data(shape, bc):
    nx, ny, nz = shape
    _say(f"case: cnn forward dyadic {shape} {bc}")
    rng = np.random.default_rng(10)
    flat = _dyadic_params(rng)
    head = rng.integers(-8, 9, (5, nz, ny, nx)) / 8.0
    with _net(shape, bc) as N:
        N.set_params(flat)
        y = N.forward(_pair(head)).cpu().numpy().astype(np.float64)
    obc = ocnn.PERIODIC if bc == "periodic" else ocnn.OUTFLOW
    ref, (_, h1, _, h2) = _oracle_forward_bf16(head, _params_from_flat(flat), obc)
    if nx * ny * nz >= 64:
        assert np.count_nonzero(h1) > 0.2 * h1.size and np.count_nonzero(h2) > 0.2 * h2.size
    assert np.array_equal(y, ref)


def test_forward_at_128_cubed_sampled_cells_bit_exact():
    # the mesh size of the learned form's benchmark: the output of a cell
    # depends only on the input within 3 cells (three 3x3x3 layers), so the
    # oracle evaluates the network on the 7^3 periodic neighbourhood of each
    # sampled cell and its centre must equal the GPU's value bit for bit
    # (dyadic data: every sum exact in FP32)
    n = 128
    shape = (n, n, n)
    rng = np.random.default_rng(21)
    flat = _dyadic_params(rng)
    head = (rng.integers(-8, 9, (5, n, n, n)) / 8.0).astype(np.float32)
    _say("case: cnn forward dyadic 128^3 periodic, sampled cells")
    with _net(shape) as N:
        N.set_params(flat)
        y = N.forward(_pair(head)).cpu().numpy().astype(np.float64)
    params = _params_from_flat(flat)
    cells = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5), (n - 1, 3, 0), (64, 64, 64)]
    cells += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(27)]
    for (k, j, i) in cells:
        idx = [np.arange(c - 3, c + 4) % n for c in (k, j, i)]
        patch = head[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]].astype(np.float64)
        ref, _ = _oracle_forward_bf16(patch, params, ocnn.PERIODIC)
        assert np.array_equal(y[:, k, j, i], ref[:, 3, 3, 3]), (k, j, i)


def test_forward_random_weights_within_fp32_accumulation_bound():
    shape = (32, 16, 12)
    nx, ny, nz = shape
    from paper_1812_07977_amd.learned import init_params
    rng = np.random.default_rng(11)
    flat = init_params(3, out_scale=1.0)
    flat[-5:] = rng.standard_normal(5)
    head = 1.0 + 0.3 * rng.standard_normal((5, nz, ny, nx))
    mu, sigma = np.full(5, 1.0), np.full(5, 0.3)
    with _net(shape) as N:
        N.set_params(flat)
        N.set_norm(mu, sigma, np.ones(5))
        y = N.forward(_pair(head)).cpu().numpy().astype(np.float64)
    # the GPU's input: (head - mu) / sigma in FP32, rounded to BF16
    h32 = head.astype(np.float32)
    x = ocnn.bf16_round(((h32 - np.float32(1.0)) * np.float32(1.0 / 0.3)).astype(np.float64))
    params = _params_from_flat(flat)
    ref, (a1, h1, a2, h2) = _oracle_forward_bf16(x, params, ocnn.PERIODIC)
    # Where an FP32 and an FP64 sum straddle a BF16 rounding boundary the two
    # sides round a hidden activation to neighbouring BF16 values, at most
    # one BF16 unit (2^-8 |h|) apart, and the difference propagates through
    # the later layers.  Bound, from absolute values: E1 = 2^-8 |h1|,
    # E2 = 2^-8 |h2| + |W2| * E1, and for y: |W3| * E2 plus the FP32
    # accumulation error of the last layer, 1e-5 of its absolute sums.
    r = ocnn.bf16_round
    w2, w3 = r(params[1][0]), r(params[2][0])
    z2, z3 = np.zeros(HIDDEN_CH), np.zeros(5)
    e1 = 2.0 ** -8 * np.abs(h1)
    e2 = 2.0 ** -8 * np.abs(h2) + ocnn.conv3(e1, np.abs(w2), z2, ocnn.PERIODIC)
    absum = ocnn.conv3(np.abs(h2), np.abs(w3), np.abs(params[2][1]), ocnn.PERIODIC)
    bound = ocnn.conv3(e2, np.abs(w3), z3, ocnn.PERIODIC) + 1e-5 * absum
    err = np.abs(y - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    # and typically far inside it
    assert np.median(err / absum) < 1e-3


@pytest.mark.parametrize("shape", [(32, 8, 8), (96, 8, 6), (32, 1, 1), (64, 3, 1),
                                   (32, 24, 48), (64, 40, 20)])
def test_gradients_match_the_oracle(shape):
    # (96, 8, 6): three 32-cell blocks per row (the weight-gradient kernel
    # takes two per step, so the second of the last pair is masked) and
    # fewer rows than workgroups (some sum nothing); (32, 1, 1) and
    # (64, 3, 1): one row or one plane, where every y or z shift wraps onto
    # the cell itself.  (32, 24, 48) and (64, 40, 20): 1152 and 800 mesh
    # rows over the 512 weight-gradient workgroups, so each workgroup sums
    # two or three rows and many of those runs cross from the last row of a
    # plane to the first row of the next
    nx, ny, nz = shape
    _say(f"case: cnn gradients {nx}x{ny}x{nz} periodic")
    from paper_1812_07977_amd.learned import split_params
    import torch
    rng = np.random.default_rng(12)
    flat = _dyadic_params(rng)
    head = rng.integers(-8, 9, (5, nz, ny, nx)) / 8.0
    with _net(shape) as N:
        N.set_params(flat)
        U = _pair(head)
        params = _params_from_flat(flat)
        y, cache = _oracle_forward_bf16(head, params, ocnn.PERIODIC)
        # a target whose error y - t is exactly representable in BF16
        e = rng.integers(-8, 9, y.shape) / 8.0
        t = (y - e).astype(np.float32)
        assert np.array_equal(t.astype(np.float64), y - e)
        loss, g = N.gradients(U, torch.from_numpy(t).cuda())
    # oracle: the loss gradient 2 e / N is exact in BF16 (N a power of 2 times
    # 5 is not, so round it as the GPU does)
    n = e.size
    dy = ocnn.bf16_round(np.float32(2.0 / n) * e.astype(np.float32))
    assert loss == pytest.approx(np.mean(e * e), rel=1e-12)
    # backward with the GPU's roundings: gradients of the hidden layers are
    # rounded to BF16 before they are used
    (w1, b1), (w2, b2), (w3, b3) = params
    r = ocnn.bf16_round
    a1, h1, a2, h2 = cache
    dw3, db3, dh2 = ocnn.conv3_backward(h2, r(w3), dy, ocnn.PERIODIC)
    da2 = r(dh2 * (h2 > 0))
    dw2, db2, dh1 = ocnn.conv3_backward(h1, r(w2), da2, ocnn.PERIODIC)
    da1 = r(dh1 * (h1 > 0))
    dw1, db1, _ = ocnn.conv3_backward(head, r(w1), da1, ocnn.PERIODIC)
    # scales: the same sums over absolute values
    aw3, ab3, _ = ocnn.conv3_backward(np.abs(h2), np.abs(r(w3)), np.abs(dy), ocnn.PERIODIC)
    aw2, ab2, _ = ocnn.conv3_backward(np.abs(h1), np.abs(r(w2)), np.abs(da2), ocnn.PERIODIC)
    aw1, ab1, _ = ocnn.conv3_backward(np.abs(head), np.abs(r(w1)), np.abs(da1), ocnn.PERIODIC)
    got = split_params(g.astype(np.float64))
    # FP32 sums over the cells: at most n u of the sum of absolute terms
    tol = 1.5 * head[0].size * 2.0 ** -24
    for name, gg, ref, sc in [("W1", got[0], dw1, aw1), ("b1", got[1], db1, ab1),
                              ("W2", got[2], dw2, aw2), ("b2", got[3], db2, ab2),
                              ("W3", got[4], dw3, aw3), ("b3", got[5], db3, ab3)]:
        err = np.abs(gg - ref)
        assert np.all(err <= tol * sc + 1e-30), (name, float(np.max(err / (sc + 1e-300))))
        assert np.max(np.abs(ref)) > 0, name


def _far_apart_cells(rng, n, count, min_sep, first=()):
    """The cells `first` followed by random cells of a periodic n^3 mesh, count
    in all, each pair more than min_sep cells apart along some axis
    (Chebyshev distance, periodic)."""
    def far(c, d):
        return max(min(abs(a - b), n - abs(a - b)) for a, b in zip(c, d)) > min_sep
    cells = list(first)
    assert all(far(c, d) for q, c in enumerate(cells) for d in cells[:q])
    while len(cells) < count:
        c = tuple(int(v) for v in rng.integers(0, n, 3))
        if all(far(c, d) for d in cells):
            cells.append(c)
    return cells


def test_gradients_at_128_cubed_sparse_target_match_oracle_patches():
    # The learned form's mesh size and launch configuration: 128^3 periodic,
    # 16384 mesh rows, so each of the 512 weight-gradient workgroups sums 32
    # rows, and the input-gradient convolutions (ReLU mask fused) march
    # 8-plane chunks.  The target equals the network output except at K
    # sampled cells, so the output gradient is zero elsewhere and every
    # parameter gradient is the sum of the samples' contributions.  A
    # sample's contribution depends only on the input within 3 cells (the
    # hidden-layer gradients reach 2 cells out, the weights they multiply 1
    # more), so the oracle evaluates the forward and backward pass on each
    # sample's 7^3 periodic neighbourhood with only its centre's output
    # gradient set.  Samples are more than 5 cells apart, so no two
    # backward footprints meet and each BF16 rounding of a hidden gradient
    # sees one sample's value, as on the GPU.
    import torch
    from paper_1812_07977_amd.learned import split_params
    n = 128
    K = 48
    rng = np.random.default_rng(22)
    flat = _dyadic_params(rng)
    head = rng.integers(-8, 9, (5, n, n, n)) / 8.0
    # the first two neighbourhoods wrap around the mesh on every axis / on two
    cells = _far_apart_cells(rng, n, K, 5, first=[(0, 0, 0), (64, n - 1, 1)])
    _say(f"case: cnn gradients 128^3 periodic, sparse target at {len(cells)} cells")
    with _net((n, n, n)) as N:
        N.set_params(flat)
        U = _pair(head)
        y = N.forward(U)
        t = y.clone()
        e = (rng.integers(1, 9, (len(cells), 5)) * rng.choice([-1, 1], (len(cells), 5)) / 8.0)
        for (k, j, i), ev in zip(cells, e):
            t[:, k, j, i] = y[:, k, j, i] - torch.from_numpy(ev.astype(np.float32)).cuda()
        loss, g = N.gradients(U, t)
        y_np = y.cpu().numpy()
        t_np = t.cpu().numpy()
    # the GPU's loss kernel: d = y - t in FP32, output gradient
    # bf16(fp32(2 / N) d), N = 5 n^3
    d = (y_np - t_np).astype(np.float32)
    nz_d = np.count_nonzero(d)
    assert 0 < nz_d <= 5 * len(cells)
    scale = np.float32(2.0 / (5 * n ** 3))
    assert loss == pytest.approx(float(np.sum(d.astype(np.float64) ** 2)) / (5 * n ** 3), rel=1e-12)
    params = _params_from_flat(flat)
    (w1, b1), (w2, b2), (w3, b3) = params
    r = ocnn.bf16_round
    sums = [np.zeros_like(a) for a in (w1, b1, w2, b2, w3, b3)]
    abss = [np.zeros_like(a) for a in (w1, b1, w2, b2, w3, b3)]
    P = ocnn.PERIODIC
    for (k, j, i) in cells:
        idx = [np.arange(c - 3, c + 4) % n for c in (k, j, i)]
        x = head[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]
        _, (a1, h1, a2, h2) = _oracle_forward_bf16(x, params, P)
        dy = np.zeros((5, 7, 7, 7))
        dy[:, 3, 3, 3] = r(scale * d[:, k, j, i])
        dw3, db3, dh2 = ocnn.conv3_backward(h2, r(w3), dy, P)
        da2 = r(dh2 * (h2 > 0))
        dw2, db2, dh1 = ocnn.conv3_backward(h1, r(w2), da2, P)
        da1 = r(dh1 * (h1 > 0))
        dw1, db1, _ = ocnn.conv3_backward(x, r(w1), da1, P)
        aw3, ab3, _ = ocnn.conv3_backward(np.abs(h2), np.abs(r(w3)), np.abs(dy), P)
        aw2, ab2, _ = ocnn.conv3_backward(np.abs(h1), np.abs(r(w2)), np.abs(da2), P)
        aw1, ab1, _ = ocnn.conv3_backward(np.abs(x), np.abs(r(w1)), np.abs(da1), P)
        for acc, v in zip(sums, (dw1, db1, dw2, db2, dw3, db3)):
            acc += v
        for acc, v in zip(abss, (aw1, ab1, aw2, ab2, aw3, ab3)):
            acc += v
    got = split_params(g.astype(np.float64))
    # FP32 sums of the nonzero terms only (adding a zero is exact): at most
    # 125 per sample (the first layer's gradient reaches 2 cells out)
    tol = 1.5 * 125 * len(cells) * 2.0 ** -24
    for name, gg, ref, sc in zip(["W1", "b1", "W2", "b2", "W3", "b3"], got, sums, abss):
        err = np.abs(gg - ref)
        assert np.all(err <= tol * sc + 1e-30), (name, float(np.max(err / (sc + 1e-300))))
        assert np.max(np.abs(ref)) > 0, name


def test_adam_step_matches_the_oracle():
    shape = (32, 8, 8)
    nx, ny, nz = shape
    import torch
    from paper_1812_07977_amd.learned import init_params
    rng = np.random.default_rng(13)
    flat = init_params(4)
    head = 1.0 + 0.2 * rng.standard_normal((5, nz, ny, nx))
    t = torch.from_numpy((0.1 * rng.standard_normal((5, nz, ny, nx))).astype(np.float32)).cuda()
    with _net(shape) as N:
        N.set_params(flat)
        U = _pair(head)
        _, g = N.gradients(U, t)
        N.train_step(U, t, 1e-3)
        new = N.get_params()
    ref, _, _ = ocnn.adam(flat.astype(np.float64), g.astype(np.float64), np.zeros(flat.size),
                          np.zeros(flat.size), 1, lr=1e-3)
    assert np.max(np.abs(new - ref)) <= 1e-6 * 1e-3 + 1e-7 * np.max(np.abs(flat))


def test_restriction_and_target_match_the_oracle():
    import torch
    rng = np.random.default_rng(14)
    fine = 1.0 + 0.5 * rng.random((5, 16, 12, 40))
    with _net((20, 6, 8)) as N:
        tau = np.array([0.5, 0.25, 2.0, 1.0, 4.0])
        N.set_norm(np.zeros(5), np.ones(5), tau)
        F = torch.from_numpy(fine).cuda()
        U = N.restrict(F)
        pair = U.cpu().numpy().astype(np.float64)
        R = ocnn.restrict2(fine)
        assert np.array_equal(pair[0], R.astype(np.float32).astype(np.float64))
        # the compensation is itself FP32: the pair holds R to about 2^-48
        assert np.max(np.abs(pair[0] - pair[1] - R)) <= 2.0 ** -46 * np.max(np.abs(R))
        # target against a perturbed plain state
        P = U.clone()
        P[0] += 0.01
        t = N.make_target(F, P).cpu().numpy().astype(np.float64)
    p = P.cpu().numpy().astype(np.float64)
    ref = (R - (p[0] - p[1])) / tau[:, None, None, None]
    assert np.max(np.abs(t - ref) / np.abs(ref)) <= 2.0 ** -23


def test_correction_applies_and_falls_back():
    import torch
    import workloads as wl
    shape = (32, 16, 8)
    nx, ny, nz = shape
    from paper_1812_07977_amd.learned import init_params, param_count
    U0 = wl.random_plane(nx, ny, nz, seed=5, v=(0.3, 0.1, 0.0))
    from paper_1812_07977_amd import Fluid
    with Fluid(shape, bc="periodic", dtype="f32") as F:
        S = F.state_from(U0)
        torch.cuda.synchronize()
    start = S.cpu().numpy().astype(np.float64)
    with _net(shape) as N:
        # all-zero network: zero correction, applied, state unchanged
        N.correct(S)
        assert N.counts() == (1, 0)
        assert np.array_equal(S.cpu().numpy(), start.astype(np.float32))
        # a real correction: the state moves, totals do not
        flat = init_params(5, out_scale=1.0)
        N.set_params(flat)
        N.set_norm(U0.mean(axis=(1, 2, 3)), U0.std(axis=(1, 2, 3)) + 1e-3, np.full(5, 1e-3))
        N.correct(S)
        assert N.counts() == (2, 0)
        after = S.cpu().numpy().astype(np.float64)
        before_v = start[0] - start[1]
        after_v = after[0] - after[1]
        change = after_v - before_v
        assert np.max(np.abs(change)) > 1e-5
        for f in range(5):
            assert abs(change[f].sum()) <= 1e-5 * np.abs(change[f]).sum()
        # a correction that empties some cells: fallback, state unchanged
        N.set_norm(U0.mean(axis=(1, 2, 3)), U0.std(axis=(1, 2, 3)) + 1e-3, np.full(5, 1e3))
        N.correct(S)
        assert N.counts() == (2, 1)
        assert np.array_equal(S.cpu().numpy().astype(np.float64), after)


def test_training_reduces_the_loss():
    import torch
    from paper_1812_07977_amd.learned import init_params
    shape = (32, 16, 16)
    nx, ny, nz = shape
    rng = np.random.default_rng(15)
    head = 1.0 + 0.2 * rng.standard_normal((5, nz, ny, nx))
    # a target that is a fixed smooth function of the input
    t = np.roll(head, 1, axis=3) - head
    with _net(shape) as N:
        N.set_params(init_params(6))
        N.set_norm(np.ones(5), np.full(5, 0.2), np.ones(5))
        U = _pair(head)
        T = torch.from_numpy(((t) / 0.2).astype(np.float32)).cuda()
        first = N.train_step(U, T, 3e-3, want_loss=True)
        for _ in range(150):
            N.train_step(U, T, 3e-3)
        last = N.train_step(U, T, 3e-3, want_loss=True)
    _say(f"training loss {first:.4e} -> {last:.4e}")
    assert last < 0.3 * first


def test_scale_aware_inputs_match_the_oracle():
    # mode 1: inputs (log rho, v, log p) from FP64 primitive recovery of the
    # head, normalised in FP32 and rounded to BF16
    import workloads as wl
    shape = (32, 16, 12)
    nx, ny, nz = shape
    from paper_1812_07977_amd.learned import init_params
    U0 = wl.random_plane(nx, ny, nz, seed=3, v=(0.4, -0.3, 0.2))
    head = U0.astype(np.float32).astype(np.float64)
    flat = init_params(7, out_scale=1.0)
    feats = ocnn.features(head, 1.4)
    mu = feats.mean(axis=(1, 2, 3))
    sigma = feats.std(axis=(1, 2, 3)) + 0.1
    with _net(shape) as N:
        N.set_params(flat)
        N.set_features(1)
        N.set_norm(mu, sigma, np.ones(5))
        y = N.forward(_pair(head)).cpu().numpy().astype(np.float64)
    f32 = feats.astype(np.float32)
    x = ocnn.bf16_round(((f32 - mu.astype(np.float32)[:, None, None, None])
                         * (1.0 / sigma).astype(np.float32)[:, None, None, None]).astype(np.float64))
    params = _params_from_flat(flat)
    ref, (a1, h1, a2, h2) = _oracle_forward_bf16(x, params, ocnn.PERIODIC)
    r = ocnn.bf16_round
    w1, w2, w3 = r(params[0][0]), r(params[1][0]), r(params[2][0])
    z32, z5 = np.zeros(HIDDEN_CH), np.zeros(5)
    # as in the random-weight test, plus one BF16 unit of the inputs (the
    # device and numpy logarithms may round a feature differently)
    e0 = 2.0 ** -8 * np.abs(x)
    e1 = 2.0 ** -8 * np.abs(h1) + ocnn.conv3(e0, np.abs(w1), z32, ocnn.PERIODIC)
    e2 = 2.0 ** -8 * np.abs(h2) + ocnn.conv3(e1, np.abs(w2), z32, ocnn.PERIODIC)
    absum = ocnn.conv3(np.abs(h2), np.abs(w3), np.abs(params[2][1]), ocnn.PERIODIC)
    bound = ocnn.conv3(e2, np.abs(w3), z5, ocnn.PERIODIC) + 1e-5 * absum
    err = np.abs(y - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert np.median(err / absum) < 1e-3


def test_committed_correction_is_the_kahan_sum_of_the_delta():
    # the state after an accepted correction, element by element: delta =
    # tau (y - mean y) rounded to FP32 (mean in FP64), Kahan-added into the
    # (head, compensation) pair in FP32, from the network output y of the
    # same state
    import math
    import torch
    import workloads as wl
    from paper_1812_07977_amd import Fluid
    from paper_1812_07977_amd.learned import init_params
    shape = (48, 20, 9)
    nx, ny, nz = shape
    U0 = wl.random_plane(nx, ny, nz, seed=17, v=(0.2, -0.1, 0.3))
    with Fluid(shape, bc="periodic", dtype="f32") as F:
        S = F.state_from(U0)
        torch.cuda.synchronize()
    tau = np.array([2e-3, 3e-3, 3e-3, 3e-3, 5e-3])
    with _net(shape) as N:
        N.set_params(init_params(9, out_scale=1.0))
        N.set_norm(U0.mean(axis=(1, 2, 3)), U0.std(axis=(1, 2, 3)) + 1e-3, tau)
        y = N.forward(S).cpu().numpy().astype(np.float64)
        before = S.cpu().numpy()
        N.correct(S)
        assert N.counts() == (1, 0)
        after = S.cpu().numpy()
    head, comp = before[0], before[1]
    for f in range(5):
        mean = math.fsum(y[f].ravel()) / y[f].size
        d = (tau[f] * (y[f] - mean)).astype(np.float32)
        yy = d - comp[f]
        s = head[f] + yy
        c2 = (s - head[f]) - yy
        assert np.array_equal(after[0][f], s), f
        assert np.array_equal(after[1][f], c2), f
    assert not np.array_equal(after, before)


@pytest.mark.parametrize("shape, clip", [((48, 20, 9), 0.0), ((70, 37, 40), 0.05)])
def test_committed_correction_with_clip_is_the_kahan_sum_of_the_delta(shape, clip):
    # mode 0 sums the network output for the mean inside the last
    # convolution: on a ragged mesh of several work items per workgroup, with
    # and without clipping, the committed state is still the Kahan sum of
    # tau (clip(y) - mean clip(y)) with y from the plain forward pass
    import math
    import torch
    import workloads as wl
    from paper_1812_07977_amd import Fluid
    from paper_1812_07977_amd.learned import init_params
    nx, ny, nz = shape
    U0 = wl.random_plane(nx, ny, nz, seed=23, v=(0.1, 0.3, -0.2))
    with Fluid(shape, bc="outflow", dtype="f32") as F:
        S = F.state_from(U0)
        torch.cuda.synchronize()
    tau = np.array([1e-3, 2e-3, 2e-3, 2e-3, 4e-3])
    with _net(shape, bc="outflow") as N:
        N.set_params(init_params(31, out_scale=1.0))
        N.set_norm(U0.mean(axis=(1, 2, 3)), U0.std(axis=(1, 2, 3)) + 1e-3, tau)
        N.set_features(0, clip)
        y = N.forward(S).cpu().numpy().astype(np.float64)
        before = S.cpu().numpy()
        N.correct(S)
        assert N.counts() == (1, 0)
        after = S.cpu().numpy()
    if clip > 0:
        assert np.mean(np.abs(y) > clip) > 0.05  # the clip is exercised
        y = np.clip(y, -clip, clip)
    head, comp = before[0], before[1]
    for f in range(5):
        mean = math.fsum(y[f].ravel()) / y[f].size
        d = (tau[f] * (y[f] - mean)).astype(np.float32)
        yy = d - comp[f]
        s = head[f] + yy
        c2 = (s - head[f]) - yy
        assert np.array_equal(after[0][f], s), f
        assert np.array_equal(after[1][f], c2), f


def test_scale_aware_targets_and_clipped_correction():
    import torch
    import workloads as wl
    from paper_1812_07977_amd import Fluid
    from paper_1812_07977_amd.learned import init_params
    shape = (16, 12, 10)
    nx, ny, nz = shape
    rng = np.random.default_rng(16)
    fine = wl.random_plane(2 * nx, 2 * ny, 2 * nz, seed=2, v=(0.3, 0.2, -0.1))
    tau = np.array([0.01, 0.02, 0.02, 0.02, 0.03])
    with _net(shape) as N:
        N.set_features(1)
        N.set_norm(np.zeros(5), np.ones(5), tau)
        F = torch.from_numpy(fine).cuda()
        U = N.restrict(F)
        U[0] *= torch.from_numpy((1.0 + 0.01 * rng.standard_normal((5, nz, ny, nx))).astype(np.float32)).cuda()
        t = N.make_target(F, U).cpu().numpy().astype(np.float64)
        p = U.cpu().numpy().astype(np.float64)
        u = p[0] - p[1]
        S = ocnn.scales(u, 1.4)
        ref = (ocnn.restrict2(fine) - u) / (tau[:, None, None, None] * S)
        assert np.max(np.abs(t - ref) / np.maximum(np.abs(ref), 1e-30)) <= 2.0 ** -20
        # correction relative to local scales, clipped at 0.5: every cell
        # moves by at most tau S 0.5 (plus the mean removal), totals stay
        N.set_params(init_params(8, out_scale=1.0))
        N.set_norm(np.array([0.0, 0.0, 0.0, 0.0, 0.0]), np.ones(5), tau)
        N.set_features(1, 0.5)
        before = U.cpu().numpy().astype(np.float64)
        N.correct(U)
        assert N.counts() == (1, 0)
        after = U.cpu().numpy().astype(np.float64)
    change = (after[0] - after[1]) - (before[0] - before[1])
    Sb = ocnn.scales(before[0].astype(np.float64), 1.4)
    lim = tau[:, None, None, None] * Sb * 0.5
    for f in range(5):
        mean_shift = tau[f] * np.max(Sb[f]) * 0.5
        assert np.all(np.abs(change[f]) <= lim[f] + mean_shift + 1e-6 * np.abs(before[0][f])), f
        assert abs(change[f].sum()) <= 1e-5 * np.abs(change[f]).sum()
    assert np.max(np.abs(change)) > 0
