/*
 * gs_fluid.h -- C ABI of libgs_fluid.so: one explicit RK2 finite-volume step
 * of the 3D ideal-gas Euler equations on a Cartesian mesh, as hand-written
 * HIP kernels for AMD gfx950 (MI355X), in FP64 or in a compensated FP32 form.
 *
 * The step is the paper's "Fluid Evolution" loop body (Section 3, Algorithms
 * 1 and 2): ComputeTimeStep, then two substeps of ComputeDifferences,
 * ComputeReconstruction, ComputeFluxes and ComputeUpdate combined as
 *     U(1)   = U(n) + dU(U(n))
 *     U(n+1) = 0.5 * (U(n) + U(1) + dU(U(1))),
 * with GhostExchange supplying two ghost layers per side before each
 * substep.  The paper names these kernels without formulas; this library
 * computes (FP64 form; the FP32 form below differs only in precision):
 *   - primitive recovery v = m/rho, p = (gamma-1)(E - m.v/2);
 *   - differences of primitives (index ranges of the paper's listing in
 *     Section 3) limited by minmod into slopes sigma; face states
 *     W_L = W_i + sigma_i/2 and W_R = W_{i+1} - sigma_{i+1}/2;
 *   - HLL fluxes with Davis signal-speed estimates from the face states;
 *   - dU = -dt * sum over axes x, y, z of (F(i+1/2) - F(i-1/2)) / h;
 *   - TimeStep = CFL / max over cells of sum_d (|v_d| + c) / h_d, a
 *     max-reduction;
 *   - ghost layers: outflow repeats the edge cell, periodic wraps.  The
 *     ghosts are virtual (index arithmetic); arrays hold proper cells only.
 *
 * Data layout.  An FP64 state U is one contiguous device array of doubles
 * [5][nz][ny][nx], x fastest, fields (rho, m_x, m_y, m_z, E) -- the paper's
 * StorageForm Value(cell, field) with cells contiguous per field (Section
 * 2.1).  Pointers must be device pointers (hipMalloc or a PyTorch tensor's
 * data_ptr()) aligned to 8 bytes (256 recommended), valid on the device that
 * was current at gs_fluid_create.  The caller owns U and keeps it alive until
 * the work queued on the handle's stream has finished.
 *
 * FP32 form (dtype GS_F32).  The state is FP32 and the reconstruction and
 * flux arithmetic runs in FP32; primitive recovery (where p = (gamma-1)(E -
 * m.v/2) cancels when the kinetic energy dominates), signal rates, the time
 * step, the device time and conserved totals are FP64.  The first substep
 * keeps its increment dU(U(n)) in the workspace beside U(1), and the second
 * adds 0.5 (dU(U(n)) + dU(U(1))) to U(n) by Kahan summation, so that
 * increments below the rounding of U are not lost.  A state is therefore a
 * pair: U points to 2 x 5 x nz x ny x nx floats,
 * the head [5][nz][ny][nx] followed by the compensation [5][nz][ny][nx], and
 * represents head - compensation (exact in FP64).  The kernels read the head
 * as the cell values; only the RK combine reads and rewrites the
 * compensation.  Start from compensation = 0, or from the FP32 rounding of
 * head - u for FP64 initial data u, which the pair then holds to about 48
 * bits.  Pointers must be aligned to 4 bytes (256 recommended).
 *
 * Streams and synchronisation.  Every call queues work on the handle's
 * stream (hipStream_t, NULL = the legacy default stream) and returns without
 * waiting, except gs_fluid_dt, gs_fluid_dt_last, gs_fluid_step_dt,
 * gs_fluid_totals, gs_fluid_sync, gs_fluid_get_time and gs_fluid_kernel_ms,
 * which wait for the stream.  A handle is not
 * thread-safe: use one handle per stream.
 *
 * Errors.  Every int-returning call returns GS_OK or a negative status;
 * arguments are validated before any HIP call, so bad arguments return
 * GS_ERR_ARG even on a machine without a GPU.  gs_fluid_last_error gives a
 * message.  Kernels never fault on bad data: a non-positive or non-finite
 * density or pressure met in any state the kernels read sets a device flag,
 * which the next waiting call reports as GS_ERR_NONPHYSICAL (once; the flag
 * is then cleared).  The affected state holds unspecified finite or NaN
 * values.
 */
#ifndef GS_FLUID_H
#define GS_FLUID_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_fluid gs_fluid;

/* Boundary kinds (GhostExchange on the physical boundary). */
enum { GS_BC_OUTFLOW = 0, GS_BC_PERIODIC = 1 };

/* Arithmetic types of the state: FP64, or the compensated FP32 form. */
enum { GS_F64 = 0, GS_F32 = 1 };

/* Status codes. */
enum {
    GS_OK = 0,
    GS_ERR_ARG = -1,          /* invalid argument; nothing was queued     */
    GS_ERR_HIP = -2,          /* HIP runtime error or no gfx950 device   */
    GS_ERR_NONPHYSICAL = -3,  /* rho or p <= 0 or not finite was met     */
    GS_ERR_STATE = -4         /* call not valid in the handle's state    */
};

/*
 * Create a solver for an nx*ny*nz mesh of proper cells (nx*ny below 2^29,
 * nx*ny*nz*5 at most 2^40) with widths dx, dy,
 * dz, ratio of specific heats gamma (> 1), Courant number cfl (0 < cfl <= 1)
 * and boundary kind bc, on the current HIP device, for states of type dtype
 * (GS_F64 or GS_F32).  stream is a hipStream_t or NULL.  Allocates the
 * handle's workspace: the first substep's result U(1) (FP32 form: with its
 * increment, 2 x 5 x nz x ny x nx floats) plus about 100 KB of reduction
 * words; the handle owns it until
 * gs_fluid_destroy.  On success *out is the handle; on failure *out is NULL
 * and gs_fluid_last_error(NULL) gives the reason.  Paper: persistent
 * device allocation at initialisation (Section 2.1, AllocateDevice), one
 * device per process (Section 1; the default device of Section 2.2).
 */
int gs_fluid_create(int nx, int ny, int nz, double dx, double dy, double dz,
                    double gamma, double cfl, int bc, int dtype, void* stream,
                    gs_fluid** out);

/*
 * ComputeTimeStep (Algorithm 1): *dt_out = cfl / max over proper cells of
 * sum_d (|v_d| + c)/h_d for state U (device, layout of the handle's dtype;
 * the FP32 form reads the head).  FP64 arithmetic in both forms.  One
 * reduction pass over U on the stream, then waits for the stream.  Returns
 * GS_ERR_NONPHYSICAL if U, or any state read since the last waiting call,
 * held a non-physical cell.
 */
int gs_fluid_dt(gs_fluid* h, const void* U, double* dt_out);

/*
 * ComputeTimeStep (Algorithm 1) without a reduction pass: *dt_out = cfl /
 * the max signal rate of the state that the handle's last gs_fluid_advance
 * or gs_fluid_step_dt wrote, which the second substep of its last step
 * computed while writing it (the max over cells is exact, so the result
 * equals gs_fluid_dt's on that unchanged state bit for bit).  Waits for the
 * stream.  GS_ERR_STATE if the last state written came from gs_fluid_step,
 * or none since the handle was created or its time was set; a caller that
 * modifies the state itself afterwards must use gs_fluid_dt instead.
 * Non-physical states are reported as by gs_fluid_dt.
 */
int gs_fluid_dt_last(gs_fluid* h, double* dt_out);

/*
 * One RK2 step (Algorithm 1, both substeps) of size dt (finite, > 0): U is
 * read as U(n) and overwritten in place with U(n+1).  Two kernel launches on
 * the stream; no host synchronisation.  The handle's device time advances by
 * dt.
 */
int gs_fluid_step(gs_fluid* h, void* U, double dt);

/*
 * The host-synchronised loop of Algorithm 1 in one call: gs_fluid_step
 * whose second substep also takes the max signal rate of U(n+1) while
 * writing it, then gs_fluid_dt_last: waits and sets *dt_next to the CFL
 * time step of U(n+1), with no reduction pass (200 instead of 240 bytes of
 * HBM traffic per cell and step).  Errors as gs_fluid_step and
 * gs_fluid_dt_last.
 */
int gs_fluid_step_dt(gs_fluid* h, void* U, double dt, double* dt_next);

/*
 * nsteps RK2 steps with the time step computed on the device: before the
 * first step a reduction pass over U; after that every step's dt comes from
 * the max-reduction fused into the previous step's second substep.  With
 * t_end > 0 each dt is clipped to t_end - t (t = the handle's device time)
 * and steps at or after t_end leave U unchanged.  dt_log, if not NULL, is a
 * device array of nsteps doubles receiving each step's dt.  No host
 * synchronisation: the paper's host round trip per step (Algorithm 2) is
 * replaced by a device-resident dt.
 */
int gs_fluid_advance(gs_fluid* h, void* U, int nsteps, double t_end,
                     double* dt_log);

/*
 * Allocation-free advance, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same computation as gs_fluid_create (with the same
 * arguments and checks) + gs_fluid_set_time(t0) + gs_fluid_advance(U, nsteps,
 * t_end, dt_log) with the default launch shape, giving bit-identical U and
 * dt_log, but without a handle: the workspace (U(1), reduction partials,
 * device words) is a 96 MiB array inside the library that each GPU it runs
 * on holds until the process ends.  Calls no hipMalloc, hipFree or other
 * allocating routine.
 *   U: caller's device state, layout of dtype (FP32: the [head | comp] pair).
 *   t_out, flags_out: optional device pointers (NULL: not written) receiving,
 *     at the end of the queued work, the device time after the last step and
 *     the non-physical flag word (bit 0 set if any state read held a
 *     non-positive or non-finite density or pressure).
 * Meshes whose workspace exceeds the array (more than 2,516,582 cells, FP64
 * or FP32) are rejected with GS_ERR_ARG before any HIP call, as are the
 * arguments gs_fluid_create or gs_fluid_advance would reject.  Asynchronous
 * on `stream`; errors are reported by gs_fluid_last_error(NULL).  The array
 * keeps the last call's contents, and every call on one GPU shares it: calls
 * whose queued work overlaps on one GPU (two host threads, or two streams
 * without ordering) race and give undefined results.
 */
int gs_fluid_advance_noalloc(int nx, int ny, int nz, double dx, double dy,
                             double dz, double gamma, double cfl, int bc,
                             int dtype, void* U, int nsteps, double t0,
                             double t_end, double* dt_log, double* t_out,
                             unsigned int* flags_out, void* stream);

/*
 * Conserved totals: totals[f] = sum over proper cells of field f of U
 * (host array of 5 doubles), for the FP32 form of head - compensation.  FP64
 * with error-free (TwoSum) accumulation in a fixed order: deterministic, and
 * within a few units of the last place of the exact sum.  A diagnostic, not
 * a step of the paper's algorithm: with periodic boundaries the
 * finite-volume update conserves these sums up to rounding, since every
 * face flux enters two cells with opposite signs.  One reduction pass on the
 * stream, then waits; reports a pending non-physical flag like gs_fluid_sync.
 */
int gs_fluid_totals(gs_fluid* h, const void* U, double* totals);

/* Wait for the stream; report a pending non-physical flag. */
int gs_fluid_sync(gs_fluid* h);

/* Device time: read (waits for the stream) or set (queued on the stream). */
int gs_fluid_get_time(gs_fluid* h, double* t_out);
int gs_fluid_set_time(gs_fluid* h, double t);

/* Change the stream used by later calls.  The new stream first waits for
 * the work already queued on the old one (an event recorded there), since
 * that work still uses the handle's workspace and device words. */
int gs_fluid_set_stream(gs_fluid* h, void* stream);

/*
 * Launch shape of the stage kernels: workgroups of 256 threads own a
 * (256/tile_y) x tile_y column tile (tile_y 8 or 16; 0 = the default, 16
 * for FP64 and 8 for FP32, rows of one 128-byte cache line per field) and
 * march chunk_z planes (>= 1; 0 = chosen from the mesh).  Results do not
 * depend on the shape.
 */
int gs_fluid_set_launch(gs_fluid* h, int tile_y, int chunk_z);

/*
 * Per-kernel timing with HIP events recorded on the handle's stream around
 * every stage-kernel launch.  kernel: 0 = first substep, 1 = second substep,
 * 2 = dt reduction.  gs_fluid_kernel_ms waits for the stream, returns the
 * summed milliseconds and the number of launches since the last call (or
 * since enabling), and resets them.
 */
int gs_fluid_profile(gs_fluid* h, int enable);
int gs_fluid_kernel_ms(gs_fluid* h, int kernel, double* total_ms, int* launches);

/* Bytes of device memory the handle allocates for a mesh (workspace). */
long long gs_fluid_workspace_bytes(int nx, int ny, int nz, int dtype);

/*
 * HBM streaming probe, the ceiling the stage kernels' bandwidth is compared
 * with (not a step of the paper's algorithm; the paper argues its kernels
 * are bound by memory bandwidth, Section 4).  Queues one kernel on stream
 * (hipStream_t or NULL) computing c[i] = a[i] (b NULL: one read per write,
 * the first substep's mix) or c[i] = a[i] + b[i] (two reads per write, the
 * second substep's mix) for i < n, FP64, in 16-byte vectors.  flags bit 0:
 * non-temporal stores.  a, b, c: device arrays of n doubles, 16-byte
 * aligned, c not overlapping a or b; n even and > 0.  Does not wait; time
 * it with events on the same stream.  Errors: GS_ERR_ARG (message from
 * gs_fluid_last_error(NULL)), GS_ERR_HIP on a failed launch.
 */
int gs_fluid_stream_probe(const double* a, const double* b, double* c, long long n,
                          int flags, void* stream);

/* Release the handle and its workspace (does not wait for the stream; the
 * caller must not destroy a handle with work in flight).  NULL: no-op. */
void gs_fluid_destroy(gs_fluid* h);

/* Last error message of the handle, or of the last failed create if h is
 * NULL.  Never NULL; "" if none. */
const char* gs_fluid_last_error(const gs_fluid* h);

#ifdef __cplusplus
}
#endif

#endif /* GS_FLUID_H */
