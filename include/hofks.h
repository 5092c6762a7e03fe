/*
 * hofks.h -- C ABI of the MI355X (gfx950) library for the High Order Fast
 * Kinetic Scheme (HOFKS) of Dimarco & Loubere, arXiv:1212.0204.
 *
 * One time step t^n -> t^{n+1} of the discrete-velocity BGK model (sections 3
 * and 4.3.1 of the paper):
 *   relaxation  f* = lambda f^n + (1 - lambda) E[U^n],  lambda = exp(-dt/tau)
 *   transport   f_K(x_j, v_k) = f*(x_j - v_k dt), an exact shift of the pieces
 *   moments     U_* = P(T(lambda f^n)),  U_M = P(T((1 - lambda) E[U^n]))  (eq. UK)
 *   Euler       U_E = (1 - lambda) MUSCL_dt(U^n)             (section 4.3.2)
 *   correction  f^{n+1} = f_K + C^T (C C^T)^{-1} (U_E - U_M)  (eq. minim_full)
 *               U^{n+1} = U_* + U_E                           (eq. mom)
 * E[U] is the conservative Maxwellian of eq. (minimMax).
 *
 * Lattice.  Velocity nodes v_k = k dv with k in {-n/2 .. n/2-1} per axis for
 * even n and {-(n-1)/2 .. (n-1)/2} for odd n; by default the library sets
 * dt = dx / dv, so v_k dt = k dx and transport moves every piece by exactly k
 * cells.  A smaller dt in the descriptor gives off-lattice transport (the
 * pieces keep their shape and move continuously; each step shifts them by a
 * whole number of cells that follows their accumulated offset).
 *
 * Layouts (host arrays).  Cells are x-fastest: j = (jz*Ny + jy)*Nx + jx.
 * Moments U are component-major, U[r*Nc + j] with r = 0 (rho), 1..d (rho u),
 * d+1 (E = |u|^2 rho/2 + d rho theta/2).  The distribution read by
 * hofks_read_f is velocity-plane major, f[k*Nc + j], velocity nodes x-fastest:
 * k = (iz*n + iy)*n + ix.
 *
 * Ownership.  The library never allocates device memory: the caller passes a
 * device workspace of at least hofks_workspace_size() bytes (for example a
 * torch uint8 tensor) and a HIP stream; both must outlive the context.  Host
 * pointers belong to the caller and are only read/written during the call.
 *
 * Errors.  Every call returns a status; nothing crosses the ABI as an
 * exception.  Kernels record non-physical states (rho <= 0, theta <= 0 or
 * non-finite moments) and sub-step overflow in a device flag that is sticky:
 * it is reported by the next synchronising call (hofks_read_*, hofks_sync).
 * hofks_last_error() gives a message for the last failing call.  A context is
 * not thread-safe.
 */
#ifndef HOFKS_H
#define HOFKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hofks_ctx hofks_ctx;

typedef enum {
  HOFKS_OK = 0,
  HOFKS_EINVAL = -1,   /* bad argument or descriptor                          */
  HOFKS_ESIZE = -2,    /* workspace or host buffer too small                  */
  HOFKS_EDEVICE = -3,  /* a HIP runtime call failed                           */
  HOFKS_ENONPHYS = -4, /* rho <= 0, theta <= 0 or non-finite moments were met */
  HOFKS_ESTATE = -5    /* call out of order, or Euler sub-step cap exceeded   */
} hofks_status;

typedef struct {
  int dim;          /* d in {1,2,3}: space and velocity dimension (section 2) */
  int n_cells[3];   /* N_x, N_y, N_z; unused axes are ignored                  */
  double dx;        /* cell size, the same on every axis (section 4)          */
  int n_vel;        /* velocity nodes per axis, >= 2                          */
  double dv;        /* velocity step; dt = dx / dv                            */
  int bc[3];        /* per axis: 0 periodic, 1 outflow (zero gradient)        */
  int precision;    /* 0: FP64 pieces; 1: FP32 pieces, FP64 compensated sums  */
  int scheme;       /* 0 HOFKS; 1 FKS (U_E := U_M); 2 HOFKS with phi == 1;
                       3 HOFKS with the WENO Euler solve (section 4.3.3:
                       WENO5 of the Lax-Friedrichs split flux, three-stage
                       SSP Runge-Kutta, CFL 0.4 instead of eq. (Time2)'s 1/2;
                       single grids only, not the closure form)              */
  double dt;        /* 0: the lattice dt = dx/dv (every piece moves k cells);
                       0 < dt <= dx/dv: off-lattice transport (section 4.2):
                       the pieces of velocity v_k sit at the accumulated
                       offset v_k n dt and a step moves them by
                       ceil(c (n+1) - 1/2) - ceil(c n - 1/2) cells,
                       c = v_k dt / dx; n_vel a multiple of 4 in 2D/3D;
                       not for batches or the closure form                   */
  int splitting;    /* 0: first order, relaxation then transport (sections
                       4.2, 4.3.1); 1: Strang, R_{dt/2} T_dt R_{dt/2} per
                       step (section 4.2): consecutive half relaxations act
                       as one (the moments are unchanged by a relaxation), so
                       the first step after the state is set relaxes by half
                       and hofks_read_f applies the last step's pending half
                       towards E[U^n]; U is the same either way.  Not for
                       batches or the closure form                           */
} hofks_grid_desc;

/* Bytes of device workspace a context with this descriptor needs. */
hofks_status hofks_workspace_size(const hofks_grid_desc *desc, size_t *bytes);

/* Create a context on the current HIP device.  dev_ws: device pointer to at
 * least hofks_workspace_size() bytes, 256-byte aligned; hip_stream: the
 * hipStream_t every kernel of this context is launched on (0 = null stream). */
hofks_status hofks_create(const hofks_grid_desc *desc, void *dev_ws,
                          size_t ws_bytes, void *hip_stream, hofks_ctx **out);

/* Relaxation time tau of eq. (B): tau > 0, tau = +INF (free transport,
 * lambda = 1) or tau = 0 (lambda = 0).  Takes effect at the next step. */
hofks_status hofks_set_tau(hofks_ctx *ctx, double tau);

/* Initial data (section 4.2): U^0 from host arrays rho[Nc], u[d*Nc]
 * (component-major), theta[Nc]; f^0 = E[U^0].  Synchronous. */
hofks_status hofks_set_state_macro(hofks_ctx *ctx, const double *rho,
                                   const double *u, const double *theta);

/* Arbitrary initial distribution f^0 (layout f[k*Nc + j], FP64 host array of
 * Nv*Nc values); U^0 = P(f^0), eq. (DM).  Synchronous. */
hofks_status hofks_set_state_f(hofks_ctx *ctx, const double *f, size_t bytes);

/* Advance n_steps >= 0 time steps; asynchronous on the context's stream: it
 * returns once the last step is queued.  In a call of more than 16 steps on
 * a 2D or 3D grid it reads back the Euler sub-step count of earlier steps
 * (waiting for a step once it is 16 behind the one being queued), so that the
 * launches of the later steps follow a count that grows during the call. */
hofks_status hofks_step(hofks_ctx *ctx, int n_steps);

/* Wait for the stream and report the sticky device flag. */
hofks_status hofks_sync(hofks_ctx *ctx);

/* Copy U^n to host U[(d+2)*Nc] (layout above).  Synchronous. */
hofks_status hofks_read_moments(hofks_ctx *ctx, double *U);

/* Copy f^n to host (layout above) as FP64 values; bytes >= 8*Nv*Nc.
 * Synchronous.  Uses the idle half of the piece buffers as staging. */
hofks_status hofks_read_f(hofks_ctx *ctx, double *f, size_t bytes);

/* Checkpoint and resume.  hofks_state_bytes gives the size of a host image
 * of the state (header with the grid, tau, step count and the speeds of U^n,
 * then U^n, the pending correction, the records and the pieces);
 * hofks_read_state fills it (synchronous; HOFKS_ESTATE while closure cells
 * hold no pieces), hofks_write_state restores it into a context of the same
 * grid (HOFKS_EINVAL otherwise), after which stepping continues exactly as
 * from the saved step.  Host buffers belong to the caller.  Not available
 * for batches. */
hofks_status hofks_state_bytes(hofks_ctx *ctx, size_t *bytes);
hofks_status hofks_read_state(hofks_ctx *ctx, void *host, size_t bytes);
hofks_status hofks_write_state(hofks_ctx *ctx, const void *host, size_t bytes);

/* Number of Euler sub-steps of the last completed step (0 if none ran) and
 * the steps taken so far.  Synchronous. */
hofks_status hofks_read_counters(hofks_ctx *ctx, int *substeps, long *steps);

/* Euler sub-steps run so far by the persistent tail of the Euler solve (the
 * sub-steps beyond the per-sub-step launches of a step; see
 * hofks_set_euler_launches), counted since the state was set.  Synchronous.
 * Always 0 for a batch. */
hofks_status hofks_read_tail_substeps(hofks_ctx *ctx, long *n);

/* The Euler solve of a step (section 4.3.2, sub-cycled) is launched as k
 * single-sub-step kernels followed by a persistent kernel that runs any
 * further sub-steps with an in-kernel barrier between them.  k = 0 (the
 * default) takes k = (sub-steps of the last step seen at a synchronising
 * call, or read back during a long hofks_step call) + 1, dropping the + 1
 * while that count is steady, and k = 1 on a 1D grid (scheme other than 3)
 * that fits one persistent block, where the barrier is the block's own;
 * k >= 1 fixes it, so that k = 1 runs every sub-step after the first in the
 * persistent kernel.  The two kernels form the same faces from the same values; their
 * results agree to rounding (the compiler may contract their products
 * differently).  HOFKS_EINVAL
 * for k < 0 or a batch. */
hofks_status hofks_set_euler_launches(hofks_ctx *ctx, int k);

/* Per-kernel timing with hipEvents recorded around each launch group of
 * hofks_step: group 0 = the Euler sub-steps (on the library's auxiliary
 * stream, beside group 1), 1 = the kinetic kernel (relaxation, shift, moment
 * sums), 2 = the per-cell update, 3 = the closure network and its indicator
 * (closure form only).  If ms/launches are non-null, synchronise and return
 * the summed elapsed milliseconds and the launch counts of each group since
 * the last call, then clear them.  enable is a bit mask of the groups to
 * record for the following steps (bit g: group g; 15 all, 0 none); each
 * recorded group adds two events per step to its stream.  HOFKS_EINVAL for
 * a mask outside 0..15. */
hofks_status hofks_kernel_timing(hofks_ctx *ctx, int enable, double ms[4],
                                 int launches[4]);

double hofks_dt(const hofks_ctx *ctx);
const char *hofks_last_error(const hofks_ctx *ctx);
void hofks_destroy(hofks_ctx *ctx);

/* ------------------------------------------------------------- batches
 * Many independent 1D-1V tubes (dim 1, outflow, precision 1, scheme 0; n_vel
 * a multiple of 8), each with its own cells, dx, velocity grid, dt = dx/dv
 * and relaxation time, advanced together: per step an Euler launch (one
 * block per tube, two tubes of at most 2048 cells per block, or one block
 * per part of a split tube) and a kinetic launch (one block per tube
 * segment) run side by side on two streams, then a per-cell update launch;
 * hofks_step replays a captured graph of consecutive steps.  The same
 * calls as above apply to a batch context with concatenated host arrays:
 *   hofks_set_state_macro  rho, u, theta of tube 0 cells, then tube 1, ...
 *   hofks_read_moments     per tube 3 x Nx_i (component-major), concatenated
 *   hofks_read_f           per tube n_vel_i x Nx_i, concatenated
 * hofks_set_tau and hofks_set_state_f return HOFKS_EINVAL for a batch.  A
 * tube that meets a non-physical state (or needs more Euler sub-steps than
 * the cap) is flagged and from then on no longer advanced (its values are
 * not meaningful; with split Euler solves its parts keep running); its flag
 * is read with hofks_batch_tube_flags and the synchronising calls still
 * succeed, so the other tubes stay readable. */
hofks_status hofks_batch_workspace_size(const hofks_grid_desc *descs, int n,
                                        size_t *bytes);
/* taus[n]: per-tube tau (> 0, +INF or 0); other arguments as hofks_create. */
hofks_status hofks_batch_create(const hofks_grid_desc *descs, const double *taus,
                                int n, void *dev_ws, size_t ws_bytes,
                                void *hip_stream, hofks_ctx **out);
/* Per-tube error bits (1 non-physical, 2 sub-step cap) to host flags[n]. */
hofks_status hofks_batch_tube_flags(hofks_ctx *ctx, int *flags);
/* Autotuner.  Times `steps` steps of each candidate launch configuration on
 * the current state, which is advanced (set the state again afterwards), and
 * keeps the fastest:
 *   single grid: wavefronts per kinetic block and piece loads issued ahead,
 *                then the placement of the Euler solve (beside the kinetic
 *                kernel on the library's second stream, or before it on the
 *                context's stream), choice = (wavefronts, loads,
 *                euler_before); 3D grids use blocks of four y rows (four
 *                wavefronts) and tune the loads only;
 *   batch:       cells per kinetic item, then the part size of the split
 *                Euler solves, choice = (cells, euler_part, 0).
 * cache_path (may be NULL) is a JSON-lines file of earlier choices keyed by
 * the grid or batch shape; a match skips the timing, a new choice is
 * appended.  choice[3] may be NULL. */
hofks_status hofks_autotune(hofks_ctx *ctx, int steps, const char *cache_path,
                            int choice[3]);

/* Set the launch configuration of a single grid without timing: wavefronts
 * per kinetic block and loads ahead as the autotuner's candidates (2D FP64
 * grids: 2 or 4 wavefronts, 4 or 8 loads; others: 2, 4 or 8 (2D/3D)
 * wavefronts, 8 or 16 loads; 3D grids 4 wavefronts), and euler_before = 1 to
 * run the Euler solve before the kinetic kernel on the context's stream
 * (0: beside it on the library's second stream).  Results do not depend on
 * the configuration.  HOFKS_EINVAL for a batch or an unavailable choice. */
hofks_status hofks_set_launch_config(hofks_ctx *ctx, int wavefronts, int loads, int euler_before);

/* Set the launch configuration of a batch without timing: cells per kinetic
 * item (256, 512 or 1024) and euler_part, the cells per part of a split Euler
 * solve (1024 or 2048: a tube of Nx > euler_part cells is solved by
 * ceil(Nx / euler_part) blocks meeting after every sub-step, when that is at
 * most 64 and at most the compute units; 0: every tube whole in one block).
 * Results do not depend on the configuration.  The work order is taken
 * again from the current speeds.  HOFKS_EINVAL for a single grid or an
 * unavailable choice. */
hofks_status hofks_batch_set_launch_config(hofks_ctx *ctx, int cells, int euler_part);

/* ------------------------------------------------- learned closure (2D-2V)
 * Not part of the paper: near-equilibrium cells skip the pieces.  The moment
 * update of eq. (UK) with (mom) splits into the transported equilibrium,
 * the Euler part U_E and the non-equilibrium term
 *   N_j = sum_k w m_k (f* - E)(j - k, k) = lambda sum_k w m_k (f - E)(j - k, k).
 * In a closure cell U^{n+1} = lambda sum_k w m_k E(j - k, k) + U_E + N^ with
 * N^ = lambda * sigma * (y - y0) (.) (rho, rho c, rho c, E)_j, y the network
 * output on the 3 x 3 stencil of U^n (37 inputs, see hofks_closure_snapshot)
 * and y0 its output on a uniform stencil.  A cell runs the full kinetic
 * step (eqs. (UK), (mom), (minim_full)) when lambda sigma max|y - y0| >
 * threshold, when its last kinetic step had lambda max|delta| / s >
 * threshold (every cell counts as such for the first step after the state
 * is set), or when such a cell lies within
 * n_vel/2 cells along each axis; kinetic cells that read an upstream closure
 * cell use its equilibrium.  Needs dim 2 and scheme 0; a step with tau = +inf
 * or 0 runs the plain scheme. */

/* Network: device pointer to hofks_mlp_packed_bytes() bytes (16-byte
 * aligned) written by hofks_mlp_pack; owned by the caller and read by every
 * following step until hofks_closure_disable.  The output on the uniform
 * stencil (y0) is evaluated at the first closure step after this call and
 * again when tau changes: weights rewritten in place take effect after
 * calling hofks_closure_enable again.  sigma scales the output;
 * threshold < 0 makes every cell kinetic, +INF every cell a closure cell
 * (up to the delta marks, also compared with it). */
hofks_status hofks_closure_enable(hofks_ctx *ctx, const void *packed_weights,
                                  double sigma, double threshold);
/* Back to the plain scheme; the next step runs every cell kinetic and
 * rebuilds the pieces of former closure cells from their equilibrium. */
hofks_status hofks_closure_disable(hofks_ctx *ctx);
/* One plain step (every cell kinetic) that also writes, for each cell j,
 * the network inputs of U^n to x[j][37] (device, FP32): for stencil cell
 * c = 3 (dy + 1) + (dx + 1) the values rho_c/rho_j - 1, (u_c - u_j)/c_j (x,
 * y), theta_c/theta_j - 1, then log10(tau/dt) clamped to [-8, 8]; and the target
 * N_j / (lambda s_j) to t[j][4] (device, FP32), s_j = (rho, rho c, rho c, E)
 * of U^n, c = sqrt(gamma theta).  Needs 1e-12 <= lambda < 1. */
hofks_status hofks_closure_snapshot(hofks_ctx *ctx, float *x, float *t);
/* Closure steps run since the state was set, and the kinetic cell-steps
 * among them.  Synchronous. */
hofks_status hofks_closure_stats(hofks_ctx *ctx, long *closure_steps,
                                 unsigned long long *kinetic_cell_steps);

/* The network, on the matrix cores: 37 -> 64 -> 64 -> 64 -> 4, tanh hidden
 * layers, BF16 weights and activations, FP32 accumulation.  FP32 parameters
 * are flat: W1[64][37] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[4][64]
 * b4[4] (weights row-major, output index first).  All pointers are device
 * pointers owned by the caller; calls are asynchronous on `stream` and
 * return HOFKS_EINVAL for bad arguments, HOFKS_EDEVICE for a failed launch. */
int hofks_mlp_nparam(void);          /* 11012 */
size_t hofks_mlp_packed_bytes(void); /* bytes of the packed form */
/* FP32 parameters -> packed BF16 form read by the kernels (16-byte aligned) */
hofks_status hofks_mlp_pack(const float *params, void *packed, void *stream);
/* y[n][4] = net(x[n][37]); y 16-byte aligned */
hofks_status hofks_mlp_forward(const void *packed, const float *x, float *y, long n,
                               void *stream);
/* grad[11012] (overwritten) and *loss of L = (1/(4n)) sum (y - t)^2 over a
 * batch of n samples, sample s being row idx[s] of x[.][37] and t[.][4]
 * (row s if idx is NULL); evaluated at the packed weights.  The sums run in a
 * fixed order (one partial per block in `work`, then the partials in block
 * order), so the result is reproducible bit for bit.  work: device scratch of
 * at least hofks_mlp_grad_work_bytes(n) bytes (at most 5.6 MB), 256-byte
 * aligned, owned by the caller; HOFKS_ESIZE if smaller. */
size_t hofks_mlp_grad_work_bytes(long n);
hofks_status hofks_mlp_grad(const void *packed, const float *x, const float *t,
                            const int *idx, long n, float *grad, float *loss,
                            void *work, size_t work_bytes, void *stream);
/* hofks_mlp_grad without a work argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc): the per-block partials go to a scratch
 * array the library holds in device memory for the life of the process,
 * GRAD_WORK_MAX = 5,668,864 bytes on every GPU it runs on (its address on
 * the current device is looked up at the first call there).  Same kernels,
 * same results, bit for bit.  The call allocates nothing; every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (on several
 * streams or host threads) race; each call overwrites every partial it
 * reads, so nothing is carried between calls.  HOFKS_EINVAL for bad
 * arguments, HOFKS_ESIZE if the work exceeds the array (it cannot for
 * n >= 1), HOFKS_EDEVICE if the address lookup or a launch fails. */
hofks_status hofks_mlp_grad_noalloc(const void *packed, const float *x, const float *t,
                                    const int *idx, long n, float *grad, float *loss,
                                    void *stream);/* One Adam step (bias-corrected, step counts from 1) on FP32 params, m, v.
 * Pack again afterwards. */
hofks_status hofks_mlp_adam(float *params, const float *grad, float *m, float *v,
                            float lr, float beta1, float beta2, float eps, int step,
                            void *stream);

/* Training of the closure network on the GPU (device pointers, caller
 * owned, asynchronous on `stream`).
 *
 * hofks_closure_prepare: from n snapshot pairs (x[n][37], t[n][4], as
 * hofks_closure_snapshot writes them) form the training set.  Per output c
 * a robust scale s_c: q_c = the k-th smallest |t_c|, k = ceil(995 n / 1000),
 * then the sample standard deviation (n - 1 divisor) of the t_c with
 * |t_c| <= q_c (at least 1e-12).  Samples with |t_c / s_c| <= clip for every c
 * are copied in their original order to x_out and (t / s) to t_out (room for
 * n rows each); scales[4] (double) and the count *kept (int) are written.
 * Every sum runs in a fixed order.  work: hofks_closure_prepare_work_bytes(n)
 * bytes, 256-byte aligned. */
size_t hofks_closure_prepare_work_bytes(long n);
hofks_status hofks_closure_prepare(const float *x, const float *t, long n, float clip,
                                   float *x_out, float *t_out, double *scales, int *kept,
                                   void *work, size_t work_bytes, void *stream);
/* The scales into the output layer: W4 row c and b4[c] times scales[c]
 * (FP32 parameters; pack again afterwards). */
hofks_status hofks_mlp_fold_scales(float *params, const double *scales, void *stream);
/* One training step: the gradient of the minibatch (as hofks_mlp_grad, rows
 * idx[0..n) of x and t), one Adam step (as hofks_mlp_adam, step counts from
 * 1) on params/m/v, and the packed BF16 form written to `packed`; the loss of
 * the minibatch at the weights before the step to *loss and the gradient to
 * grad.  work as for hofks_mlp_grad. */
hofks_status hofks_closure_train_step(float *params, float *m, float *v, void *packed,
                                      const float *x, const float *t, const int *idx, long n,
                                      float lr, float beta1, float beta2, float eps, int step,
                                      float *grad, float *loss, void *work, size_t work_bytes,
                                      void *stream);
/* Network of the closure steps of a grid context: the packed weights
 * (hofks_mlp_packed_bytes() bytes, device, caller owned, 16-byte aligned)
 * read by every following closure step; the output on the uniform stencil
 * is evaluated again at the next closure step.  HOFKS_ESIZE for another
 * size.  (hofks_closure_enable also sets them, with the scale and threshold.) */
hofks_status hofks_closure_set_weights(hofks_ctx *ctx, const void *packed, size_t bytes);

/* Measurement aid: stream `bytes` (a multiple of 16, 16-byte aligned device
 * pointers) with the 16-byte non-temporal loads and stores of the piece
 * loops and no arithmetic: mode 0 reads src (dst: a 4-byte device word that
 * is written only for one improbable value), 1 writes dst, 2 copies src to
 * dst.  Asynchronous on `stream`; the caller times it.  This is the
 * reachable bandwidth the kinetic kernels are compared with, besides the
 * vendor peak. */
hofks_status hofks_stream_probe(int mode, const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HOFKS_H */
