/*
 * otfs.h -- C ABI of libotfs: LMMSE equalisation of Zak-OTFS frames by conjugate gradient
 * with the structured-sparse delay-Doppler channel applied on the fly, on one MI355X.
 *
 * The operation (paper Sec. III-B, Eq. eq_lin_sys and Eq. lmmse; Sec. IV-C, Algorithm 1):
 * for every frame, given the received DD frame y (M*N complex values), the P dominant
 * paths of the effective channel (Eq. heff_model) and the noise variance lam, compute
 *     x_hat = (H^H H + lam I)^{-1} H^H y
 * by conjugate gradient from x = 0, where H is the MN x MN DD channel matrix of Eq. Hdd.
 * H is never formed: each iteration applies H and H^H through the structured-sparse
 * gather of Eqs. sparse_mvm / sparse_herm_mvm, with the column map of Eq. map_chMatDD_col,
 * the inverse map of Eq. herm_mapping and the twisted phase of Sec. IV-B ("Phase
 * correction and coefficient synthesis").
 *
 * Conventions shared by every entry point:
 *  - Frame layout: complex64 interleaved (re, im) -- the layout of torch.complex64 -- in
 *    vector order q = l*M + k: delay bin k in [0, M) fastest, Doppler bin l in [0, N)
 *    (Sec. IV-B indexes rows this way).  A batch is the concatenation of its frames in
 *    descriptor order; total_elems = sum of M_f * N_f.
 *  - Paths: signed bin shifts, |delay| < M, |doppler| < N, i.e. (k_p - K0, l_p - L0) with the
 *    pilot reference already subtracted.  Paths of one frame may repeat a bin.
 *  - Ownership: the caller owns every device buffer (inputs, outputs, workspace, server
 *    pool).  The library never calls hipMalloc or hipFree.  All device work is enqueued
 *    on the caller's stream (a hipStream_t passed as void*, NULL = default stream) and is
 *    asynchronous; the caller keeps buffers alive until that stream completes.
 *  - Errors: every function returns an otfs_status; no C++ exception crosses the ABI.
 *    Argument errors are found on the host before anything is enqueued and return
 *    OTFS_E_INVAL; otfs_last_error() then holds a readable message (per thread).
 *    Numerical trouble in one frame never fails a batch: it is reported in that frame's
 *    otfs_frame_stats.status.  A HIP runtime error returns OTFS_E_DEVICE.
 *  - Thread safety: distinct plans / servers may be used from distinct threads.  One
 *    plan must not be used by two threads at once.
 */
#ifndef OTFS_H_
#define OTFS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OTFS_OK = 0,
  OTFS_E_INVAL = 1,        /* bad argument (detected on the host, nothing enqueued)        */
  OTFS_E_NOMEM = 2,        /* host allocation failed, or a caller buffer is too small       */
  OTFS_E_DEVICE = 3,       /* HIP runtime error                                             */
  OTFS_E_BUDGET = 4,       /* a single frame can never fit the server's memory budget       */
  OTFS_E_AGAIN = 5,        /* otfs_poll: the frame is not finished yet                      */
  OTFS_E_NOTFOUND = 6,     /* unknown ticket                                                */
  OTFS_E_UNSUPPORTED = 7,  /* a valid request this build does not handle                    */
  OTFS_E_STATE = 8         /* call out of order (e.g. plan used before otfs_plan_bind)     */
} otfs_status;

/* Text of the last non-OK status returned on the calling thread ("" if none). */
const char* otfs_last_error(void);

/* Provenance of this build: "source_sha=<16 hex digits> arch=<gfx target>", the SHA-256
 * prefix of the sources and headers the library was compiled from (static string). */
const char* otfs_build_info(void);

/* ------------------------------------------------------------------------------------ */
/* Frames, options, statistics                                                           */
/* ------------------------------------------------------------------------------------ */

/* One frame: DD grid M x N and its dominant paths (Eq. heff_model; the threshold set of
 * Eq. heff_thres with gains h_p = h_eff[k_p, l_p]).  Host pointers, read during the call
 * that receives the descriptor and not kept. */
typedef struct {
  int32_t M, N;             /* delay bins >= 1, Doppler bins >= 1, M*N <= 2^28             */
  int32_t P;                /* number of paths, 1 <= P <= 64                                */
  const float* h;           /* 2*P floats: complex gain h_p as (re, im)                      */
  const int32_t* delay;     /* P signed delay shifts tau_p,   |tau_p| < M                   */
  const int32_t* doppler;   /* P signed Doppler shifts nu_p,  |nu_p|  < N                   */
  float noise_var;          /* lam = sigma^2 >= 0: R_n = lam I (Sec. IV-C, Algorithm 1)      */
  int32_t qam;              /* square QAM size for hard decisions (4,16,64,256) or 0 = none  */
} otfs_frame_desc;

/* Option flags. */
enum {
  OTFS_D_STORED_BF16 = 1u << 0,  /* store D_{p,q} (Eq. D_definition) as bf16 (re, im) pairs
                                    in the workspace (the SS table of Eq. ds_repr) instead of
                                    synthesising it on the fly                               */
  OTFS_Y_BF16 = 1u << 1,         /* y_dev holds 2*total_elems bf16 values (re, im) instead of
                                    complex64                                                */
  OTFS_USE_GRAPH = 1u << 2,      /* otfs_lmmse_cg replays a captured hipGraph of its launch
                                    sequence (re-captured when buffers or stream change);
                                    needs a created stream, not the NULL stream             */
  OTFS_TIME_KERNEL = 1u << 3,    /* bracket the fused CG kernel with hipEvents on the caller's
                                    stream; read with otfs_plan_kernel_ms                    */
  OTFS_AGENT_BARRIER = 1u << 4,  /* fused kernel: one work queue and device-wide coherent
                                    per-frame barriers, independent of workgroup placement
                                    (default: frames stay on one XCD, barriers coherent
                                    through that XCD's L2)                                   */
  OTFS_NO_LDS_RESIDENT = 1u << 5, /* solve small one-tile frames with their vectors in memory
                                    too (default: in LDS when 5*M*N*8 bytes fit 40 KiB)      */
  OTFS_SPLIT_DIRECTION = 1u << 6, /* always form the direction p = c + beta p in a pass of its
                                    own before the H pass.  By default, when every frame
                                    gathered straight from memory has P <= 8 (and no stored
                                    D), the H pass forms it inside its gathers instead; the
                                    results are identical                                   */
  OTFS_LDS_GATHER = 1u << 8,     /* fused kernel: frames of several tiles whose rows split
                                    into 16-byte pairs (M a multiple of 128) gather H and H^H
                                    through LDS windows (each strip's source window copied in
                                    once, then read by every path) where the window fits
                                    160 KiB; the results are identical to the direct gathers */
  OTFS_D_STORED_C64 = 1u << 7    /* store D_{p,q} (Eq. D_definition) in complex64 in the
                                    workspace: the SS table of Eq. ds_repr as the paper keeps
                                    it (Sec. IV-B, "Efficient Data Structure"), P x total_elems
                                    entries of 8 bytes, built on the device at bind from the
                                    FP32 delay-ramp and wrap tables.  Excludes
                                    OTFS_D_STORED_BF16                                        */
};

/* CG options (Algorithm 1 with a per-frame stop test added in front of the direction
 * update: stop when sqrt(||c_xi||^2 / ||c_0||^2) <= rel_tol, or when xi = max_iters). */
typedef struct {
  int32_t max_iters;        /* >= 1; Algorithm 1 fixes 10                                   */
  float rel_tol;            /* >= 0; 0 runs exactly max_iters iterations                    */
  int32_t refresh_every;    /* k >= 0: every k iterations replace the recursive residual by
                               c = H^H (y - H x) - lam x computed in FP64; 0 = never         */
  uint32_t flags;           /* OTFS_* flags above                                           */
} otfs_cg_opts;

enum {
  OTFS_FRAME_RUNNING = 0,
  OTFS_FRAME_CONVERGED = 1,   /* relative residual <= rel_tol (or H^H y = 0)                */
  OTFS_FRAME_CAPPED = 2,      /* max_iters reached                                          */
  OTFS_FRAME_NONFINITE = 3,   /* a NaN/Inf appeared; x_hat holds the last finite iterate    */
  OTFS_FRAME_BREAKDOWN = 4,   /* Re(p^H a_p) <= 0; x_hat holds the last iterate             */
  OTFS_FRAME_TIMEOUT = 5,     /* an in-kernel wait exceeded its limit (should not happen)    */
  OTFS_FRAME_DRYRUN = 6       /* server created on device -1: scheduled only, no arithmetic  */
};

/* Per-frame result, written to device memory by the solver (16 bytes). */
typedef struct {
  int32_t iters;            /* number of x updates performed                                */
  float rel_res;            /* sqrt(||c||^2 / ||c_0||^2) at the last iteration              */
  int32_t status;           /* OTFS_FRAME_*                                                  */
  int32_t tiles;            /* workgroups that cooperated on the frame                      */
} otfs_frame_stats;

/* ------------------------------------------------------------------------------------ */
/* Batch plan                                                                            */
/* ------------------------------------------------------------------------------------ */
typedef struct otfs_plan otfs_plan_t;

/* Validate a batch of frames and precompute, on the host, everything the kernels need:
 * ragged offsets, per-path delay phase ramps R_p[k] = h_p e^{j 2 pi nu_p (k - tau_p)/(MN)}
 * and the wrap factors e^{j 2 pi l / N} (the twisted phase of Sec. IV-B reduced exactly,
 * in integer arithmetic, before one FP64 sincos and a rounding to FP32), and the tiling
 * of frames into workgroups.  No device work.  nframes >= 0; frames may be NULL when
 * nframes == 0.  opts may be NULL (max_iters 50, rel_tol 1e-6, no refresh, no flags).
 * On success *out owns a new plan (free with otfs_plan_free). */
otfs_status otfs_plan(const otfs_frame_desc* frames, int32_t nframes, const otfs_cg_opts* opts,
                      otfs_plan_t** out);

/* Device workspace the plan needs (bytes, 256-byte aligned start required) and the batch
 * length in complex elements.  Either output pointer may be NULL. */
otfs_status otfs_plan_workspace_bytes(const otfs_plan_t* plan, size_t* bytes,
                                      int64_t* total_elems);

/* Attach caller-owned device memory of at least otfs_plan_workspace_bytes() bytes and
 * upload the plan's tables with copies enqueued on `stream` (and, with
 * OTFS_D_STORED_BF16, build D on the device).  Selects the device that is current on
 * the calling thread.  May be called again with another workspace. */
otfs_status otfs_plan_bind(otfs_plan_t* plan, void* workspace_dev, size_t workspace_bytes,
                           void* stream);

otfs_status otfs_plan_free(otfs_plan_t* plan);

/* Frames, elements and the launch shape chosen for the fused kernel. */
typedef struct {
  int32_t nframes;
  int64_t total_elems;
  int32_t grid;             /* workgroups of the fused CG launches (summed over launches)   */
  int32_t block;            /* threads per workgroup                                        */
  int32_t max_paths;        /* largest P in the batch                                       */
  int32_t tile_elems;       /* target elements per workgroup tile                           */
  int32_t groups;           /* work-queue groups of the fused launch (XCDs, or 1)           */
  int32_t xcd_local;        /* 1: frames stay on one XCD (see OTFS_AGENT_BARRIER)           */
  int32_t lds_bytes;        /* dynamic LDS per workgroup of the fused launch (0: none)       */
  int32_t staged_frames;    /* frames whose gathers are staged through LDS windows          */
  int32_t resident_frames;  /* one-workgroup frames solved with all CG vectors in LDS       */
  int32_t launches;         /* fused-kernel launches per solve: one per kind of frame        */
  int32_t fused_direction_frames; /* frames whose H pass forms the direction in its gathers */
} otfs_plan_info_t;
otfs_status otfs_plan_info(const otfs_plan_t* plan, otfs_plan_info_t* info);

/* Change the tiling (target elements per workgroup tile, >= 1, or 0 for the built-in
 * rule) and the workgroup cap of the fused kernel (0 = occupancy limit).  Takes effect at
 * the next otfs_plan_bind.  Used by the autotuner. */
otfs_status otfs_plan_set_tiling(otfs_plan_t* plan, int32_t tile_elems, int32_t max_grid);

/* Windowed gathers: frames whose delay bins divide into strips of strip_cols columns (a
 * multiple of 64 dividing 512) and whose paths number at most 16 are tiled into such strips
 * over all Doppler rows; every gather pass streams each source row once through an LDS ring
 * chunk_rows output rows at a time and gathers every path from there.  0 turns it off (the
 * default).  Takes effect at the next otfs_plan_bind; frames outside the form's limits keep
 * row bands. */
otfs_status otfs_plan_set_window(otfs_plan_t* plan, int32_t strip_cols, int32_t chunk_rows);

/* LDS budget per workgroup for staging the gather windows of H and H^H (Eqs. sparse_mvm,
 * sparse_herm_mvm), in bytes, at most 65536; takes effect at the next otfs_plan_bind.  A
 * staged frame's workgroup copies the source rows and columns a block of its outputs can
 * reach (for c and the old p at once in the direction pass) straight from memory into
 * LDS, then does every path's gather from there; frames whose smallest window pair
 * exceeds the budget gather straight from memory.  Default 0 (off): on the measured
 * workloads direct gathers were faster.  Small one-tile frames solved resident in LDS
 * (see OTFS_NO_LDS_RESIDENT) do not depend on this budget. */
otfs_status otfs_plan_set_staging(otfs_plan_t* plan, int32_t lds_bytes);

/* ------------------------------------------------------------------------------------ */
/* Operator applications (Eq. sparse_mvm and Eq. sparse_herm_mvm), every frame of the   */
/* bound batch in one launch.  x_dev / y_dev: total_elems complex64 each, distinct.       */
/* ------------------------------------------------------------------------------------ */
otfs_status otfs_apply_H(const otfs_plan_t* plan, const void* x_dev, void* y_dev, void* stream);
otfs_status otfs_apply_HH(const otfs_plan_t* plan, const void* y_dev, void* x_dev, void* stream);

/* ------------------------------------------------------------------------------------ */
/* LMMSE by conjugate gradient (Algorithm 1), all frames of the bound batch.              */
/* ------------------------------------------------------------------------------------ */
/* Fused form: one persistent launch (per kind of frame) runs every frame's iteration loop;
 * frames are split into row tiles, the workgroups of one frame meet at per-frame barriers,
 * and each frame stops on its own.  With refresh_every = k the loop is cut after every k-th
 * iteration into segments, and two launches between segments form the FP64 true residual
 * c = H^H (y - H x) - lam x; frames of the windowed-pairs kind (OTFS_LDS_GATHER) whose LDS
 * windows fit form it inside the fused launch instead, and when every frame is of that kind
 * and the path tables are the host's, a solve is one launch.  The fused launches expect the
 * GPU to themselves: a frame's
 * tiles must all be resident at once, and work from other streams that keeps some of them
 * waiting makes the frame report OTFS_FRAME_TIMEOUT after the wait bound.  y_dev: total_elems complex64 (bf16 pairs with OTFS_Y_BF16);
 * xhat_dev: total_elems complex64 output; sym_dev: total_elems uint8 hard decisions
 * i_I * sqrt(Q) + i_Q (Eq. demod; nullable; frames with qam = 0 are left untouched);
 * stats_dev: nframes otfs_frame_stats (nullable). */
otfs_status otfs_lmmse_cg(otfs_plan_t* plan, const void* y_dev, void* xhat_dev, uint8_t* sym_dev,
                          otfs_frame_stats* stats_dev, void* stream);

/* Plain form of the same computation: one frame at a time, four unfused kernel launches
 * per iteration (H; H^H + lam + dot; update + norm; direction), scalars kept on the
 * device, the same stop rule, no FP64 refresh.  The baseline the fused form is measured
 * against. */
otfs_status otfs_lmmse_cg_plain(otfs_plan_t* plan, const void* y_dev, void* xhat_dev,
                                uint8_t* sym_dev, otfs_frame_stats* stats_dev, void* stream);

/* ------------------------------------------------------------------------------------ */
/* Discrete Zak transform (the receiver's front end)                                      */
/* ------------------------------------------------------------------------------------ */
/* DZT of nframes received time-domain frames (Sec. III-A, Eq. zak):
 *     Y[k, l] = N^{-1/2} sum_{i=0}^{N-1} y[k + i M] e^{-j 2 pi i l / N},
 * computed as the batched complex GEMM of Sec. IV-A (Eq. zak_gemm): per frame the N x M
 * matrix of samples (row i = slot, column k = delay) is multiplied by the N x N kernel
 * e^{-j 2 pi l i / N} / sqrt(N) on the matrix cores (FP32 MFMA, FP32 accumulation).  The
 * kernel is the unitary one of Eq. zak; the printed kernel matrix of Eq. zak_exp differs
 * from it by the factor sqrt(N) (-1)^l.  inverse != 0 computes Eq. iZak instead.
 * in_dev: nframes * M * N complex64, frame after frame, sample i*M + k; out_dev: the same
 * size, DD frames in vector order q = l*M + k (for the inverse the roles swap).  Distinct
 * buffers; 1 <= N <= 8192. */
otfs_status otfs_dzt(int32_t M, int32_t N, int32_t nframes, const void* in_dev, void* out_dev,
                     int32_t inverse, void* stream);

/* ------------------------------------------------------------------------------------ */
/* Bits and bit errors (Eq. demod: decided symbols demapped to bits)                      */
/* ------------------------------------------------------------------------------------ */
/* Bit errors of hard decisions against the transmitted symbol indices, per frame.  The
 * bits of a square-QAM index i_I * sqrt(Q) + i_Q are a reflected Gray code per axis
 * (g = i XOR (i >> 1), log2 sqrt(Q) bits each, in-phase bits first; the paper leaves the
 * map unspecified).  sym_dev, sym_tx_dev: total_elems uint8; errs_dev: nframes uint64
 * (overwritten); frames with qam = 0 get 0. */
otfs_status otfs_bit_errors(const otfs_plan_t* plan, const uint8_t* sym_dev,
                            const uint8_t* sym_tx_dev, uint64_t* errs_dev, void* stream);

/* The fused solve run one iteration per launch, recording after every iteration the bit
 * errors of the current estimates' decisions against sym_tx_dev: errs_dev[(xi - 1) *
 * nframes + f] for xi = 1 .. max_iters (a frame that stopped keeps its final decisions).
 * This is the measurement behind the BER-driven iteration budget of Sec. IV-C (Eq.
 * ber_convergence).  The results (x_hat, decisions, stats) are those of otfs_lmmse_cg.
 * sym_dev is required (it holds the decisions of the last recorded iteration). */
otfs_status otfs_lmmse_cg_trace(otfs_plan_t* plan, const void* y_dev, void* xhat_dev,
                                uint8_t* sym_dev, otfs_frame_stats* stats_dev,
                                const uint8_t* sym_tx_dev, uint64_t* errs_dev, void* stream);

/* ------------------------------------------------------------------------------------ */
/* Channel from a pilot frame                                                             */
/* ------------------------------------------------------------------------------------ */
/* Replace every frame's paths, on the device, by the dominant paths estimated from its
 * received pilot frame (Sec. III "Channel estimation", Sec. IV-A "Hadamard product",
 * Sec. IV-B "Dominant path determination"): the pilot is one impulse at
 * (K0, L0) = (M/2, N/2); the effective channel is estimated on the received grid as
 * h[k, l] = Y[k, l] e^{-j 2 pi K0 (l - L0) / (MN)} (Eqs. heff_exp, heff_hadamard), bin (k, l)
 * standing for the path (tau, nu) = (k - K0, l - L0); the paths are the bins with
 * |h| > theta (Eq. heff_thres; tested as |h|^2 > theta^2 in FP32 on h rounded to FP32), in
 * vector order q = l*M + k, gain h_p = h[k_p, l_p].  The first P of them are kept, P being
 * the path count given for that frame at otfs_plan (its capacity; the given paths are
 * only placeholders then).  The plan's path tables, delay-ramp tables (and, with a stored
 * D, the SS table) are rebuilt on the device; the next otfs_apply_* / otfs_lmmse_cg* calls
 * on the stream use them, with no host round trip.  The plan must be bound; frames with
 * LDS-staged or windowed gathers return OTFS_E_UNSUPPORTED.
 * ypilot_dev: total_elems complex64, one received pilot frame per frame, in batch layout;
 * theta >= 0 (the paper uses 0.08); npaths_dev: nframes int32 receiving the number of
 * bins above theta per frame (may exceed the capacity), nullable. */
otfs_status otfs_plan_paths_from_pilot(otfs_plan_t* plan, const void* ypilot_dev, float theta,
                                       int32_t* npaths_dev, void* stream);

/* The fused form for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation).  Binds the plan to the
 * library's static scratch on the current device (a workspace of at most 64 MiB, one copy
 * per GPU, held until the process ends), then runs otfs_lmmse_cg: same kernels, same
 * results.  Calls no hipMalloc / hipFree.  The caller still passes y, x_hat, the
 * decisions and the stats.  A plan whose otfs_plan_workspace_bytes() exceeds 64 MiB
 * returns OTFS_E_NOMEM; OTFS_USE_GRAPH or OTFS_TIME_KERNEL return OTFS_E_UNSUPPORTED.
 * Every call rebinds the plan (table uploads on `stream`, then a synchronisation of it).
 * All calls on one GPU share the scratch: calls that overlap in time on one GPU race, and
 * the plan stays bound to the scratch afterwards. */
otfs_status otfs_lmmse_cg_noalloc(otfs_plan_t* plan, const void* y_dev, void* xhat_dev,
                                  uint8_t* sym_dev, otfs_frame_stats* stats_dev, void* stream);

/* Read back the paths a frame currently has on the device (after otfs_plan_bind or
 * otfs_plan_paths_from_pilot): *P receives the path count; the first min(P, capacity)
 * paths' delay, Doppler and gain h_p (2 floats, re/im, read from the FP32 delay-ramp table
 * the kernels use: exact for delays >= 0, within FP32 rounding otherwise) are written to
 * the host arrays, in the order the kernels sum them.  Synchronises `stream`. */
otfs_status otfs_plan_get_paths(const otfs_plan_t* plan, int32_t frame, int32_t capacity,
                                int32_t* P, int32_t* delay, int32_t* doppler, float* h,
                                void* stream);

/* Bound of the fused kernel's in-kernel waits (per-frame barriers and neighbour waits), in
 * microseconds: a wait that is not satisfied within it gives up, raises the launch-wide
 * abort word (every other wait of the launch then gives up too), and the frames concerned
 * report OTFS_FRAME_TIMEOUT; every workgroup still exits normally.  wait_us < 0 restores
 * the default (20 s); 0 gives up at the first unsatisfied poll (for tests of that path).
 * Takes effect at the next otfs_lmmse_cg call. */
otfs_status otfs_plan_set_wait_limit(otfs_plan_t* plan, int64_t wait_us);

/* Duration in milliseconds of the launch sequence of the last otfs_lmmse_cg call that ran
 * with OTFS_TIME_KERNEL (its fused launches and, with the refresh, any refresh launches
 * between them; waits for its end event). */
otfs_status otfs_plan_kernel_ms(otfs_plan_t* plan, float* ms);

/* ------------------------------------------------------------------------------------ */
/* Serving: continuous batching of frames that arrive over time.                          */
/* ------------------------------------------------------------------------------------ */
typedef struct otfs_server otfs_server_t;

/* Start a server on `device`.  pool_dev / pool_bytes: caller-owned device memory that
 * bounds the CG state of admitted frames (the HBM admission budget); a fixed control
 * region at its start holds the step descriptors.  A scheduler thread admits queued
 * frames in arrival order while their state fits the pool, runs steps of `step_iters`
 * (>= 1) CG iterations over all admitted frames in one fused launch, and retires frames as
 * they finish; frames that arrive meanwhile join at the next step, so their work overlaps
 * on the device with frames already in flight.  A frame's tiling depends only on its own
 * shape, so its result is the same alone or among others.  opts as for otfs_plan (NULL =
 * defaults; the bf16 flags are not supported here).  device = -1 starts a dry-run server
 * that schedules and completes frames without any device work (x_hat = 0, status
 * OTFS_FRAME_DRYRUN), for testing admission on hosts without a GPU; pool_dev is then
 * not touched.  The server copies y, x_hat and the decisions through host buffers that it
 * page-locks and keeps per size for reuse (plain memory if page-locking fails); they are
 * released by otfs_server_free, so the host memory held grows with the largest number of
 * frames in flight at once. */
otfs_status otfs_server_create(int device, void* pool_dev, size_t pool_bytes,
                               const otfs_cg_opts* opts, int32_t step_iters,
                               otfs_server_t** out);

/* Queue one frame; y_host (M*N complex64, host memory) is copied before returning.
 * OTFS_E_BUDGET if the frame's state can never fit the pool; OTFS_E_DEVICE once the server
 * has failed (see otfs_last_error). */
otfs_status otfs_submit(otfs_server_t* srv, const otfs_frame_desc* frame, const void* y_host,
                        uint64_t* ticket);

/* OTFS_E_AGAIN until the frame is done; then copies x_hat (M*N complex64), decisions
 * (M*N uint8, nullable) and stats (nullable) to host memory, returns the latency from
 * submit to completion in nanoseconds (nullable) and forgets the ticket. */
otfs_status otfs_poll(otfs_server_t* srv, uint64_t ticket, void* xhat_host, uint8_t* sym_host,
                      otfs_frame_stats* stats, uint64_t* latency_ns);

/* Batched forms for front ends that hand over bursts of frames (one lock and one call for
 * many frames; the per-frame rules are those of otfs_submit and otfs_poll).
 * otfs_submit_many queues frames[0..n) with y_host[i] the received frame of frames[i], in
 * order, and writes their tickets; if any frame is rejected nothing is queued and the
 * status is that frame's.  otfs_poll_many looks up tickets[0..n): status[i] is OTFS_OK (the
 * results of ticket i were copied to xhat_host[i], sym_host[i], stats[i], latency_ns[i] and
 * the ticket is forgotten), OTFS_E_AGAIN (still running), OTFS_E_NOTFOUND or OTFS_E_DEVICE;
 * ndone counts the OTFS_OK entries.  xhat_host, sym_host, stats, latency_ns and their
 * entries are nullable like otfs_poll's arguments; status is required. */
otfs_status otfs_submit_many(otfs_server_t* srv, const otfs_frame_desc* frames, int32_t n,
                             const void* const* y_host, uint64_t* tickets);
otfs_status otfs_poll_many(otfs_server_t* srv, const uint64_t* tickets, int32_t n,
                           void* const* xhat_host, uint8_t* const* sym_host,
                           otfs_frame_stats* stats, uint64_t* latency_ns, int32_t* status,
                           int32_t* ndone);

/* Pool bytes one frame of this shape holds while admitted (frame_bytes, nullable) and the
 * size of the server's fixed control region at the start of the pool (control_bytes,
 * nullable): a pool of control_bytes + n * frame_bytes admits n such frames at once. */
otfs_status otfs_server_frame_bytes(otfs_server_t* srv, const otfs_frame_desc* frame,
                                    size_t* frame_bytes, size_t* control_bytes);

typedef struct {
  uint64_t submitted, completed, steps;
  uint64_t queued, active;          /* frames waiting for admission / holding pool memory */
  uint64_t pool_bytes_in_use, pool_bytes_peak;
  /* scheduler time, cumulative ns: enqueueing admission copies; steps from descriptor
   * building to their synchronisation (ns_gpu of it between the first and last launch on
   * the device); result copies and retirement */
  uint64_t ns_admit, ns_step, ns_gpu, ns_fetch;
} otfs_server_stats_t;
otfs_status otfs_server_stats(otfs_server_t* srv, otfs_server_stats_t* out);

/* Tile size (elements per workgroup band) for frames of shape M x N submitted from now
 * on; 0 restores the built-in rule (32768).  A frame's tiling depends only on its own
 * shape, so its result is the same alone and among other frames.  Used to apply the
 * autotuner's per-shape serving tiles. */
otfs_status otfs_server_set_tiling(otfs_server_t* srv, int32_t M, int32_t N, int32_t tile_elems);

/* Stop the scheduler (frames still queued or running are dropped) and free host state. */
otfs_status otfs_server_free(otfs_server_t* srv);

#ifdef __cplusplus
}
#endif

#endif /* OTFS_H_ */
