/*
 * gs_batch.h -- C ABI of the batched form in libgs_fluid.so: many
 * independent problems of the Euler step (include/gs_fluid.h), each with
 * its own mesh, boundary state and device time step, advanced together by
 * one launch per substep, replayed as a captured HIP graph per step.  Not in
 * the paper, whose fluid example is one problem per MPI rank (Section 4);
 * this is a form that serves many small problems on one GPU.
 *
 * Problem i has nx_i x ny_i x nz_i proper cells of width 1/max(n_i) (an
 * isotropic cell, the reading used for non-cubic meshes), the batch's gamma,
 * CFL number, boundary kind and dtype, and a caller-owned device state in the
 * layout of gs_fluid.h for that dtype (FP64 [5][nz][ny][nx]; FP32 pair).  The
 * state pointers are fixed at creation (the captured graphs hold them); the
 * caller keeps them alive until gs_batch_destroy.
 *
 * Each step is two launches (substep 1, substep 2 with the fused per-problem
 * max-reduction of the next time step): the workgroups of a persistent grid
 * draw (problem, tile, z-chunk) items from per-XCD device counters that
 * reset themselves at the end of each launch; a problem advanced in a batch
 * and alone with the same launch shape gives bit-identical results.  Work
 * runs on a stream of the handle, ordered after and before the caller's
 * stream with events; calls on one handle must not overlap.  Status codes are
 * the GS_* codes of gs_fluid.h.
 */
#ifndef GS_BATCH_H
#define GS_BATCH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_batch gs_batch;

/*
 * A batch of count problems: dims is a host array [count][3] of (nx, ny, nz)
 * (each >= 1, (nx+15)*ny below 2^29), states a host array of count device
 * pointers (aligned to 16
 * bytes).  Allocates, per problem, a workspace (one state of the dtype, FP32:
 * with the first increment) and the per-problem device words; for FP64, where
 * nx is not a multiple of 16, the workspace and a working copy of the state
 * have rows padded to whole 128-byte lines (nx rounded up to 16 doubles).
 */
int gs_batch_create(int count, const int* dims, double gamma, double cfl, int bc, int dtype,
                    void* const* states, void* stream, gs_batch** out);

/* Launch shape for every problem: tile_y 8 or 16 (0: 16 for FP64, 8 for
 * FP32) and chunk_z planes per work item (0: chosen per problem). */
int gs_batch_set_launch(gs_batch* h, int tile_y, int chunk_z);

/*
 * Autotuner: times each candidate launch shape (tile_y in {16, 8} x chunk_z
 * in {16, 32, 64}) over a few steps on scratch copies of the states (the
 * states and times are not touched), keeps the fastest, and reports it.  If
 * cache_path is not NULL, a line keyed by a hash of the batch (dtype,
 * boundary kind, gamma, CFL and every problem's mesh) is looked up there
 * first; a hit is used without timing (*from_cache = 1) and a miss is
 * appended after timing.  Waits.
 */
int gs_batch_autotune(gs_batch* h, const char* cache_path, int* tile_y, int* chunk_z,
                      int* from_cache);

/*
 * nsteps steps of every problem, each with its own device time step (CFL
 * condition of its own state), clipped to t_end if t_end > 0 (problems at
 * or past t_end stay unchanged).  use_graph != 0: each step is one replay
 * of a captured graph of the two substep launches; 0: the same launches
 * issued directly.  Before the first step, one reduction pass per problem
 * and (FP64 with padded rows) one launch that copies the caller states into
 * the working copies; after the last, one launch that copies them back (so
 * every tile row of the steps lies on whole cache lines).  The caller's
 * states must not be changed while the call's work is queued.  No host
 * wait.
 */
int gs_batch_advance(gs_batch* h, int nsteps, double t_end, int use_graph);

/* Device time of every problem (host array of count doubles); waits;
 * GS_ERR_NONPHYSICAL if any problem read a non-physical cell since the last
 * waiting call (reported once). */
int gs_batch_times(gs_batch* h, double* times);

int gs_batch_sync(gs_batch* h);
void gs_batch_destroy(gs_batch* h);
const char* gs_batch_last_error(const gs_batch* h);

#ifdef __cplusplus
}
#endif

#endif /* GS_BATCH_H */
