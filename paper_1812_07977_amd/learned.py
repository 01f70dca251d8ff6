"""Learned-correction form: Python view of the network kernels in
libgs_fluid.so (include/gs_cnn.h).

`CorrectionNet` marshals torch tensors into the C ABI; the network, its
training and the correction of a state run in the library's kernels.  A
coarse state is an FP32-form pair (torch float32, shape (2, 5, nz, ny, nx));
fine states are float64 (5, 2nz, 2ny, 2nx).
"""
import ctypes

import numpy as np

from . import _lib
from . import GSError, NonPhysicalError, OUTFLOW, PERIODIC, _stream_ptr  # noqa: F401

_BC = {"outflow": OUTFLOW, "periodic": PERIODIC, OUTFLOW: OUTFLOW, PERIODIC: PERIODIC}

HIDDEN = 32
FIELDS = 5
TAPS = 27
SHAPES = [(HIDDEN, FIELDS, 3, 3, 3), (HIDDEN,), (HIDDEN, HIDDEN, 3, 3, 3), (HIDDEN,),
          (FIELDS, HIDDEN, 3, 3, 3), (FIELDS,)]


def _check(status, handle=None):
    if status == _lib.GS_OK:
        return
    msg = _lib.lib().gs_cnn_last_error(handle).decode(errors="replace")
    if status == _lib.GS_ERR_NONPHYSICAL:
        raise NonPhysicalError(status, msg)
    raise GSError(status, msg)


def param_count():
    return _lib.lib().gs_cnn_param_count()


def split_params(flat):
    """The flat parameter vector as [W1, b1, W2, b2, W3, b3] views."""
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    return out


def init_params(seed, out_scale=0.1):
    """He-normal weights (std sqrt(2 / fan_in)) for the ReLU layers, the
    output layer scaled by out_scale, zero biases; float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, s in enumerate(SHAPES):
        if len(s) == 1:
            parts.append(np.zeros(s, dtype=np.float32))
            continue
        fan_in = s[1] * TAPS
        w = rng.standard_normal(s) * np.sqrt(2.0 / fan_in)
        if k == 4:
            w *= out_scale
        parts.append(w.astype(np.float32))
    return np.concatenate([p.ravel() for p in parts])


class CorrectionNet:
    """The 5 -> 32 -> 32 -> 5 correction network for an nx*ny*nz coarse mesh."""

    def __init__(self, shape, bc="periodic", gamma=1.4, stream=None):
        nx, ny, nz = (int(n) for n in shape)
        if bc not in _BC:
            raise ValueError(f"unknown boundary kind {bc!r}")
        self.shape = (nx, ny, nz)
        self.bc = _BC[bc]
        self.mode, self.clip = 0, 0.0
        h = ctypes.c_void_p()
        _check(_lib.lib().gs_cnn_create(nx, ny, nz, self.bc, float(gamma), _stream_ptr(stream),
                                        ctypes.byref(h)))
        self._h = h

    def _handle(self):
        if self._h is None:
            raise RuntimeError("CorrectionNet is closed")
        return self._h

    def _ptr(self, t, dtype, shape):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
            raise TypeError(f"expected a {dtype} GPU tensor")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"expected a contiguous tensor of shape {shape}")
        return ctypes.c_void_p(t.data_ptr())

    def _coarse(self, U):
        import torch
        nx, ny, nz = self.shape
        return self._ptr(U, torch.float32, (2, 5, nz, ny, nx))

    def _field(self, y):
        import torch
        nx, ny, nz = self.shape
        return self._ptr(y, torch.float32, (5, nz, ny, nx))

    def _fine(self, F):
        import torch
        nx, ny, nz = self.shape
        return self._ptr(F, torch.float64, (5, 2 * nz, 2 * ny, 2 * nx))

    # -- parameters -----------------------------------------------------------
    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != param_count():
            raise ValueError("wrong parameter count")
        h = self._handle()
        _check(_lib.lib().gs_cnn_set_params(h, a.ctypes.data_as(ctypes.c_void_p)), h)

    def get_params(self):
        a = np.empty(param_count(), dtype=np.float32)
        h = self._handle()
        _check(_lib.lib().gs_cnn_get_params(h, a.ctypes.data_as(ctypes.c_void_p)), h)
        return a

    def set_norm(self, mu, sigma, tau):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (mu, sigma, tau)]
        P = ctypes.POINTER(ctypes.c_double)
        h = self._handle()
        _check(_lib.lib().gs_cnn_set_norm(h, *[a.ctypes.data_as(P) for a in arrs]), h)
        self._norm = arrs

    def set_features(self, mode, clip=None):
        """0: conserved inputs, absolute corrections; 1: scale-aware inputs
        (log rho, v, log p) and corrections relative to local scales.  clip >
        0 clamps the applied normalised output to [-clip, clip] (None keeps
        the current value)."""
        if clip is None:
            clip = self.clip
        h = self._handle()
        _check(_lib.lib().gs_cnn_set_features(h, int(mode), float(clip)), h)
        self.mode, self.clip = int(mode), float(clip)

    # -- kernels --------------------------------------------------------------
    def forward(self, U):
        import torch
        nx, ny, nz = self.shape
        y = torch.empty((5, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = self._handle()
        _check(_lib.lib().gs_cnn_forward(h, self._coarse(U), self._field(y)), h)
        return y

    def restrict(self, fine):
        import torch
        nx, ny, nz = self.shape
        U = torch.empty((2, 5, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = self._handle()
        _check(_lib.lib().gs_cnn_restrict(h, self._fine(fine), self._coarse(U)), h)
        return U

    def make_target(self, fine, U):
        import torch
        nx, ny, nz = self.shape
        t = torch.empty((5, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = self._handle()
        _check(_lib.lib().gs_cnn_make_target(h, self._fine(fine), self._coarse(U), self._field(t)), h)
        return t

    def gradients(self, U, target):
        g = np.empty(param_count(), dtype=np.float32)
        loss = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_cnn_gradients(h, self._coarse(U), self._field(target),
                                           g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)), h)
        return loss.value, g

    def train_step(self, U, target, lr, want_loss=False):
        loss = ctypes.c_double()
        h = self._handle()
        _check(_lib.lib().gs_cnn_train_step(h, self._coarse(U), self._field(target), float(lr),
                                            ctypes.byref(loss) if want_loss else None), h)
        return loss.value if want_loss else None

    def correct(self, U):
        h = self._handle()
        _check(_lib.lib().gs_cnn_correct(h, self._coarse(U)), h)

    def counts(self):
        a, f = ctypes.c_int(), ctypes.c_int()
        h = self._handle()
        _check(_lib.lib().gs_cnn_counts(h, ctypes.byref(a), ctypes.byref(f)), h)
        return a.value, f.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            import torch
            torch.cuda.synchronize()
            _lib.lib().gs_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# data, training and evaluation (orchestration over the kernels above and
# the solver of gs_fluid.h; periodic unit cubes)
# ---------------------------------------------------------------------------

def _solvers(n, gamma, cfl):
    from . import Fluid
    fine = Fluid((2 * n,) * 3, gamma=gamma, cfl=cfl, bc="periodic", dtype="f64")
    coarse = Fluid((n,) * 3, gamma=gamma, cfl=cfl, bc="periodic", dtype="f32")
    return fine, coarse


def _advance_to(F, U, t_end, chunk=2, limit=64):
    """Advance the fine solve F (device dt) to t_end in chunks of `chunk`
    steps until its device time reaches t_end.  Steps past t_end take dt = 0
    and leave the state unchanged, but each still costs a full step, so a
    fixed generous step count would mostly compute nothing."""
    for _ in range(limit):
        F.advance(U, chunk, t_end)
        if not F.time < t_end:
            return
    raise RuntimeError(f"fine solve did not reach t = {t_end} in {chunk * limit} steps")


def generate_samples(net, fine_states, steps, gamma=1.4, cfl=0.5, stride=1):
    """Training pairs from fine FP64 runs.  For each initial fine state (a
    float64 GPU tensor (5, 2n, 2n, 2n)) and each of `steps` coarse steps: the
    coarse state R(fine) takes one plain FP32 step of the coarse CFL time step
    dt; the fine solve advances to the same time; the target is R(fine) minus
    the plain-step state.  Every stride-th step is kept.  Returns (inputs, raw
    targets): lists of GPU tensors, the pairs after the plain step and the
    unscaled corrections.  The net's normalisation must have tau = 1 while
    this runs."""
    n = net.shape[0]
    inputs, targets = [], []
    for U0 in fine_states:
        F, C = _solvers(n, gamma, cfl)
        Uf = U0.clone()
        t = 0.0
        for k in range(steps):
            Uc = net.restrict(Uf)
            dt = C.dt(Uc)
            C.step(Uc, dt)
            F.time = t
            _advance_to(F, Uf, t + dt)
            t += dt
            if k % stride == stride - 1:
                inputs.append(Uc)
                targets.append(net.make_target(Uf, Uc))
        F.close()
        C.close()
    return inputs, targets


def input_features(head, mode, gamma=1.4):
    """The network's inputs before normalisation, for statistics: the
    conserved fields (mode 0) or (log rho, v, log p) (mode 1) of a head
    (5, ...) tensor, in FP64."""
    import torch
    h = head.double()
    if mode == 0:
        return h
    rho = h[0]
    v = h[1:4] / rho
    p = (gamma - 1.0) * (h[4] - 0.5 * rho * (v * v).sum(dim=0))
    return torch.stack([torch.log(rho), v[0], v[1], v[2], torch.log(p)])


def normalisation(inputs, targets, mode=0, gamma=1.4):
    """Per-input mean and standard deviation of the plain-step states'
    features and standard deviation of the raw corrections (targets made
    with tau = 1), over all samples."""
    import torch
    feats = torch.stack([input_features(u[0], mode, gamma) for u in inputs])
    mu = feats.mean(dim=(0, 2, 3, 4)).cpu().numpy()
    sigma = feats.std(dim=(0, 2, 3, 4)).cpu().numpy()
    del feats
    tg = torch.stack(targets)
    tau = tg.double().std(dim=(0, 2, 3, 4)).cpu().numpy()
    sigma = np.maximum(sigma, 1e-3 * np.maximum(np.abs(mu), 1e-12))
    tau = np.maximum(tau, 1e-12)
    return mu, sigma, tau


# The 48 symmetries of the cube: an axis permutation and a sign per axis.
# The Euler step is symmetric under each (cells map to cells, the momentum
# components permute and change sign with their axes), so every training
# pair maps to another valid pair.
SYMMETRIES = [(perm, signs)
              for perm in [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
              for signs in [(sx, sy, sz) for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]]


def transform(A, sym):
    """Apply a cube symmetry to a state-shaped tensor (..., 5, nz, ny, nx)
    (a coarse pair or a target): reflect the axes with sign -1, then permute
    the axes so that new axis d is old axis perm[d]; the momentum fields
    follow.  Meshes must be cubic."""
    import torch
    perm, signs = sym
    lead = A.dim() - 4
    spatial = [lead + 3, lead + 2, lead + 1]          # dims of x, y, z
    out = A
    flips = [spatial[d] for d in range(3) if signs[d] < 0]
    if flips:
        out = out.flip(flips)
    order = list(range(A.dim()))
    for d in range(3):
        order[spatial[d]] = spatial[perm[d]]
    out = out.permute(order)
    idx = [0] + [1 + perm[d] for d in range(3)] + [4]
    sgn = torch.tensor([1.0] + [float(signs[perm[d]]) for d in range(3)] + [1.0],
                       dtype=A.dtype, device=A.device)
    out = out.index_select(lead, torch.tensor(idx, device=A.device))
    shape = [1] * A.dim()
    shape[lead] = 5
    return (out * sgn.view(shape)).contiguous()


def train(net, inputs, targets, iters, lr=1e-3, seed=0, log_every=0, augment=True):
    """Adam on randomly drawn samples (each under a random cube symmetry if
    augment), learning rate decayed by cosine to 10% of lr.  Targets must
    already be divided by tau.  Returns the loss history [(iteration, loss)]
    at log_every."""
    import math
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(iters):
        k = int(rng.integers(len(inputs)))
        U, T = inputs[k], targets[k]
        if augment:
            sym = SYMMETRIES[int(rng.integers(len(SYMMETRIES)))]
            U, T = transform(U, sym), transform(T, sym)
        a = lr * (0.1 + 0.9 * 0.5 * (1.0 + math.cos(math.pi * it / max(iters, 1))))
        want = bool(log_every) and (it % log_every == 0 or it == iters - 1)
        loss = net.train_step(U, T, a, want_loss=want)
        if want:
            hist.append((it, loss))
    return hist


def fit_blend(net, fine_states, steps, alphas=(0.25, 0.5, 0.75, 1.0), gamma=1.4, cfl=0.5):
    """The factor alpha that scales the applied correction: the one with the
    smallest mean L1 error after `steps` corrected steps over the given
    trajectories (validation problems, not trained on, give an honest
    choice); alpha = 0 (no correction: the plain coarse
    solve) may be listed.  Sets the net's tau to alpha tau (alpha = 0 keeps
    tau and returns 0: the caller then skips the correction) and returns
    (alpha, {alpha: error})."""
    mu, sigma, tau = net._norm
    errs = {}
    for a in alphas:
        if a == 0:
            e = [np.mean(evaluate(net, U, steps, gamma, cfl, with_net=False)["l1_plain"])
                 for U in fine_states]
            errs[a] = float(np.mean(e))
            continue
        net.set_norm(mu, sigma, a * tau)
        e = [np.mean(evaluate(net, U, steps, gamma, cfl)["l1_corrected"]) for U in fine_states]
        errs[a] = float(np.mean(e))
    best = min(errs, key=errs.get)
    net.set_norm(mu, sigma, (best if best > 0 else 1.0) * tau)
    return best, errs


def evaluate(net, fine_state, steps, gamma=1.4, cfl=0.5, with_net=True, every=0):
    """Runs the coarse FP32 solve from R(fine_state) for `steps` steps on the
    time grid of its own plain run, with and (for comparison) without the
    correction, beside the fine FP64 solve; returns a dict with the relative
    L1 errors [density, momentum, energy] of both against R(fine) at the end
    (and their means every `every` steps under "history"), the number of
    fallbacks, and the final time."""
    import torch
    n = net.shape[0]
    F, C = _solvers(n, gamma, cfl)
    Uf = fine_state.clone()
    plain = net.restrict(Uf)
    corr = plain.clone()
    a0, f0 = net.counts()
    t = 0.0
    hist = []
    for k in range(steps):
        dt = C.dt(plain)
        C.step(plain, dt)
        if with_net:
            C.step(corr, dt)
            net.correct(corr)
        F.time = t
        _advance_to(F, Uf, t + dt)
        t += dt
        if every and (k + 1) % every == 0:
            e = _errors(net, Uf, plain, corr if with_net else None)
            hist.append((k + 1, float(np.mean(e["l1_plain"])),
                         float(np.mean(e.get("l1_corrected", [0.0])))))
    out = {"time": t}
    out.update(_errors(net, Uf, plain, corr if with_net else None))
    a1, f1 = net.counts()
    out["fallbacks"], out["applied"] = f1 - f0, a1 - a0
    if every:
        out["history"] = hist
    F.close()
    C.close()
    torch.cuda.synchronize()
    return out


def _errors(net, Uf, plain, corr):
    """Relative L1 errors of the plain (and corrected) coarse states against
    R(Uf), as [density, momentum, energy]: sum |R - U| / sum |R| over the
    cells for density and energy, and for the momentum the same over all
    three components together (so that a component that is nearly zero
    everywhere does not turn small absolute errors into large relative
    ones).  Differences come from the make_target kernel with tau = 1 in
    mode 0."""
    saved = getattr(net, "_norm", None)
    mode = getattr(net, "mode", 0)
    net.set_features(0, getattr(net, "clip", 0.0))
    net.set_norm(np.zeros(5), np.ones(5), np.ones(5))
    Rv = net.restrict(Uf)
    r = (Rv[0].double() - Rv[1].double()).abs().sum(dim=(1, 2, 3)).cpu().numpy()
    groups = [(0,), (1, 2, 3), (4,)]

    def l1(U):
        d = net.make_target(Uf, U).double().abs().sum(dim=(1, 2, 3)).cpu().numpy()
        return np.array([d[list(g)].sum() / r[list(g)].sum() for g in groups])

    out = {"l1_plain": l1(plain).tolist()}
    if corr is not None:
        out["l1_corrected"] = l1(corr).tolist()
    net.set_features(mode)
    if saved is not None:
        net.set_norm(*saved)
    return out
