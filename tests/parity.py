"""Helpers shared by the GPU parity tests: running the same seeded input
through the oracle (CPU) and the HIP library (GPU) and comparing them."""
import numpy as np

import oracle

GAMMA = 1.4
CFL = 0.5
BC = {"outflow": oracle.OUTFLOW, "periodic": oracle.PERIODIC}


# A field whose reference maximum is below this fraction of the largest
# field maximum is zero in exact arithmetic and carries only the oracle's
# rounding (the transverse momenta of a flow along one axis: a face flux of
# such a component is p (S_R - S_L) / (S_R - S_L) plus rounding): it is
# measured against the largest field, as an identically zero field is.
ZERO_FIELD = 1e-10


def _field_scales(ref, per_field):
    big = max(per_field)
    return [s if s > ZERO_FIELD * big else big for s in per_field]


def rel_linf(gpu, ref):
    """Per-field max |gpu - ref| / max |ref|; a field whose reference is zero
    up to rounding (below ZERO_FIELD of the largest field maximum) is scaled
    by the largest field maximum instead."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    scales = _field_scales(ref, [float(np.max(np.abs(ref[f]))) for f in range(ref.shape[0])])
    return [float(np.max(np.abs(gpu[f] - ref[f])) / scales[f]) for f in range(ref.shape[0])]


def to_gpu(U):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).to("cuda")


def to_cpu(T):
    import torch
    torch.cuda.synchronize()
    return T.cpu().numpy()


def oracle_run(U0, bc, nsteps, t_end=0.0, spacing=None):
    U = U0.copy()
    nz, ny, nx = U.shape[1:]
    if spacing is None:
        h = 1.0 / max(nx, ny, nz)
        spacing = (h, h, h)
    dts = oracle.run(U, spacing, GAMMA, CFL, BC[bc], nsteps, t_end)
    return U, dts


def gpu_run_host_dt(U0, bc, nsteps, launch=None):
    """dt from gs_fluid_dt, then gs_fluid_step, nsteps times."""
    from paper_1812_07977_amd import Fluid
    nz, ny, nx = U0.shape[1:]
    U = to_gpu(U0)
    dts = []
    with Fluid((nx, ny, nz), gamma=GAMMA, cfl=CFL, bc=bc) as F:
        if launch:
            F.set_launch(*launch)
        for _ in range(nsteps):
            dt = F.dt(U)
            dts.append(dt)
            F.step(U, dt)
        F.sync()
        out = to_cpu(U)
    return out, np.array(dts)


def gpu_run_device_dt(U0, bc, nsteps, t_end=0.0, launch=None):
    """gs_fluid_advance: dt on the device; returns (U, dts, final time)."""
    import torch
    from paper_1812_07977_amd import Fluid
    nz, ny, nx = U0.shape[1:]
    U = to_gpu(U0)
    log = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
    with Fluid((nx, ny, nz), gamma=GAMMA, cfl=CFL, bc=bc) as F:
        if launch:
            F.set_launch(*launch)
        F.advance(U, nsteps, t_end, log)
        t = F.time
        out = to_cpu(U)
        dts = log.cpu().numpy()[:nsteps]
    return out, dts, t


# ---------------------------------------------------------------------------
# the FP32 form: states are (head, compensation) pairs; results are compared
# as head - compensation in FP64
# ---------------------------------------------------------------------------

def f32_run(U0, bc, nsteps, mode="device", dts=None, launch=None, t_end=0.0):
    """Runs the FP32 form from FP64 initial data U0.  mode "device":
    gs_fluid_advance; "host": gs_fluid_dt + gs_fluid_step per step; "given":
    gs_fluid_step with the dt sequence dts.  Returns (U as FP64 numpy,
    dts, final device time, (head, compensation) as numpy float32)."""
    import torch
    from paper_1812_07977_amd import Fluid
    nz, ny, nx = U0.shape[1:]
    with Fluid((nx, ny, nz), gamma=GAMMA, cfl=CFL, bc=bc, dtype="f32") as F:
        if launch:
            F.set_launch(*launch)
        S = F.state_from(U0)
        if mode == "device":
            log = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
            F.advance(S, nsteps, t_end, log)
            out_dts = log.cpu().numpy()[:nsteps]
        elif mode == "host":
            out_dts = []
            for _ in range(nsteps):
                dt = F.dt(S)
                out_dts.append(dt)
                F.step(S, dt)
            out_dts = np.array(out_dts)
        else:
            for dt in dts:
                F.step(S, float(dt))
            out_dts = np.asarray(dts)
        t = F.time
        out = to_cpu(F.to_f64(S))
        pair = to_cpu(S)
    return out, out_dts, t, pair


def rel_l1(gpu, ref):
    """Per-field sum |gpu - ref| / sum |ref| (a field that is zero up to
    rounding, as in rel_linf, scaled by the largest field sum)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    peaks = [float(np.max(np.abs(ref[f]))) for f in range(ref.shape[0])]
    sums = [float(np.sum(np.abs(ref[f]))) for f in range(ref.shape[0])]
    big = max(sums)
    zero = [p <= ZERO_FIELD * max(peaks) for p in peaks]
    return [float(np.sum(np.abs(gpu[f] - ref[f])) / (big if zero[f] else sums[f]))
            for f in range(ref.shape[0])]
