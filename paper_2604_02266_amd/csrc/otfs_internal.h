// Internal declarations shared by the device code (kernels.hip) and the host library
// (plan.cpp, server.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "otfs.h"

namespace otfs {

#ifndef OTFS_BLOCK
#define OTFS_BLOCK 512
#endif
constexpr int kBlock = OTFS_BLOCK;   // threads per workgroup of every kernel
constexpr int kWaves = kBlock / 64;  // wave64
#ifndef OTFS_ROWS
#define OTFS_ROWS 4
#endif
#ifndef OTFS_STRIP_LANES
#define OTFS_STRIP_LANES 64
#endif
// Lanes across one row of a band in the gather passes: OTFS_STRIP_LANES (a multiple of 64),
// doubled while the band is too short to give every thread OTFS_ROWS rows, at most a
// workgroup, and at most `width` (the lanes a whole row needs).  The host uses it to size
// the LDS windows of the windowed paired gathers.
__host__ __device__ inline int strip_lanes_rule(int width, int band_rows) {
  int t = OTFS_STRIP_LANES;
  while (t < kBlock && t * band_rows < kBlock * OTFS_ROWS) t <<= 1;
  return width < t ? width : t;
}

// Coefficients D_{p,q}: synthesised on the fly from the delay-ramp and wrap tables, or read
// from a stored P x E table (the SS representation of Eq. ds_repr) in bf16 or complex64.
constexpr int kDNone = 0, kDBf16 = 1, kDC64 = 2;
constexpr int kMaxPathsDev = 64;   // largest P of a frame
inline int stored_mode(uint32_t flags) {
  return (flags & OTFS_D_STORED_C64) ? kDC64 : ((flags & OTFS_D_STORED_BF16) ? kDBf16 : kDNone);
}

// Per-frame CG scalars that persist between launches of the fused kernel (a serving step
// ends in the middle of a frame's iteration loop and the next step resumes it).
struct FrameState {
  int32_t iter;      // iterations completed
  int32_t status;    // OTFS_FRAME_*
  int32_t pbuf;      // which direction buffer (p0 / p1) holds the current p
  int32_t pending;   // 1: x += alpha p and p = c + beta p still to be applied
  float cn;          // ||c||^2 of the current residual
  float cn0;         // ||c_0||^2 = ||H^H y||^2
  float alpha;       // step of the last iteration (pending x update)
  float beta;        // cn_new / cn_old of the last iteration (pending direction update)
  float rel;         // sqrt(cn / cn0)
  int32_t init;      // 1 once b = H^H y has been formed
  float cn_hist[2];  // plain form: ||c||^2 by iteration parity
  int32_t refresh;   // 1: left the fused launch for the FP64 refresh (x already updated)
};

// Everything a kernel needs to know about one frame.  Built on the host, uploaded once
// per bind.  Vector pointers address device memory (the plan workspace or a server slot).
struct FrameDev {
  const void* y;          // received frame (complex64, or bf16 pairs with OTFS_Y_BF16)
  float2* x;              // estimate
  uint8_t* sym;           // hard decisions (nullable)
  otfs_frame_stats* stats;// per-frame stats (nullable)
  float2* c;              // residual
  float2* p0;             // direction, double-buffered
  float2* p1;
  float2* t;              // H p
  float2* a;              // H^H H p + lam p
  float2* u;              // the refresh's residual y - Hx, formed in FP64, kept in FP32 (nullable)
  const float2* rtab;     // P x M: R_p[k] = h_p e^{j 2 pi nu_p (k - tau_p) / (MN)}
  const float2* wtab;     // N: W[l] = e^{j 2 pi l / N}
  const double2* rtab64;  // FP64 copies of the two tables for the refresh (nullable)
  const double2* wtab64;
  const int2* paths;      // P x (tau_p, nu_p)
  const void* dtab;       // stored D_{p,q}, P x E, bf16 pairs or complex64 (nullable)
  float* part_pa;         // T partial sums of Re(p^H a)
  float* part_cc;         // T partial sums of ||c||^2
  double* part_d;         // T FP64 partial sums (refresh)
  unsigned* bar;          // arrival counter of the per-frame barrier
  unsigned* prog;         // T per-tile counters: phases whose rows the neighbours may gather
  FrameState* st;
  int64_t off;            // element offset of the frame inside batch-wide buffers
  int32_t M, N, P, T;     // grid, paths, workgroup tiles
  float lam;
  float qscale;           // sqrt(2 (Q - 1) / 3) rounded to FP32
  int32_t qside;          // sqrt(Q), 0 = no decisions
  int32_t flags;
  int32_t max_iters;
  float tol;
  int32_t refresh_every;
  int32_t index;          // frame index in its batch (stats slot)
  // LDS staging of the gathers (0 = gather straight from memory): column chunk and row
  // sub-band of one staged block, and the delay / Doppler shift ranges of the paths
  int32_t skc, ssb, swin;   // swin: LDS elements per staged vector (window, padded)
  // LDS-windowed paired gathers (staged kind, 0 = off): strip columns of the window's
  // owner strips and the window's width in columns (even; M + 2 when it spans the rows)
  int32_t lpk, lwc, lwr;   // ... and its height in rows (for the tallest band)
  int32_t tau_lo, tau_hi, nu_lo, nu_hi;
  // 1: a one-workgroup frame whose five CG vectors (x, c, p, t, a) live in LDS for the
  // whole solve (y read once, x written once)
  int32_t resident;
  // 1: the H pass of the split form stores t with the non-temporal policy (large frames,
  // whose vectors overflow L2 anyway); smaller frames keep t in L2 for the H^H gathers
  int32_t stream_t;
  // windowed gathers (0 = off): the frame's tiles are strips of win_w delay columns over
  // all Doppler rows, and each gather pass streams the source rows through an LDS window
  // win_rc output rows at a time
  int32_t win_w, win_rc;
  // path capacity: the P given at otfs_plan; a path table estimated on the device from a
  // pilot frame (otfs_plan_paths_from_pilot) may set P to anything in [0, pcap]
  int32_t pcap;
};

// One workgroup's share of one frame: Doppler rows [l_begin, l_end) of delay columns
// [k_begin, k_end) (row bands span every column; windowed strips span every row).
struct WorkItem {
  int32_t frame;
  int32_t tile;
  int32_t l_begin;
  int32_t l_end;
  int32_t k_begin;
  int32_t k_end;
};

// Windowed gathers: paths held in registers per thread (frames with more paths use the
// other launch kinds), and 64-element row pieces each wave stages per chunk.
constexpr int kWinPaths = 16;
constexpr int kWinLoads = 6;
// LDS bytes of a frame's window: (2 rc + d_nu) rows x (w + d_tau) complex64 columns,
// with d_nu, d_tau the Doppler and delay shift ranges of its paths (both widened to 0)
inline int win_lds_bytes(int w, int rc, int dtau, int dnu) {
  return (2 * rc + dnu) * (w + dtau) * 8;
}

// Batch-wide buffers passed to a launch.  A null base means "use the per-frame pointer
// in FrameDev" (server slots); otherwise the frame's data lives at base + off.
struct Bases {
  const void* y;
  float2* x;
  uint8_t* sym;
  otfs_frame_stats* stats;
};

// ---- launchers (kernels.hip) -----------------------------------------------------------
constexpr int kMaxGroups = 16;   // work-queue groups (one per XCD in XCD-local mode)
#ifndef OTFS_STAGE_ROWS
#define OTFS_STAGE_ROWS 2
#endif
constexpr int kStageRows = OTFS_STAGE_ROWS;   // output rows per thread in one staged block
constexpr int kDefaultStageBytes = 0;           // LDS per workgroup for staged windows (off)
constexpr int kResidentBytes = 40 * 1024;       // LDS of a frame solved resident in LDS
constexpr int kStageVecs = 2;    // vectors staged at once (phase A stages c and the old p)

// One workgroup per item.  in/out are batch-wide complex64 buffers (frame at base + off).
// lds_bytes: dynamic LDS for staged windows (0 if no frame is staged).
hipError_t launch_apply(bool adjoint, int sd, const FrameDev* frames, const WorkItem* items,
                        int nitems, const float2* in, float2* out, int lds_bytes, hipStream_t s);

// Reset barrier counters and CG state of frames [0, nframes), the abort word and the
// queue cursors of ngroups groups.
hipError_t launch_reset(const FrameDev* frames, int nframes, unsigned* abort_flag,
                        unsigned* qhead, int ngroups, hipStream_t s);

// Serving step preamble: clear barrier counters, queue cursors and abort word, mark stats
// slots running; keeps the frames' CG state.
hipError_t launch_step_reset(const FrameDev* frames, int nframes, unsigned* abort_flag,
                             unsigned* qhead, int ngroups, hipStream_t s);

// Fused persistent CG over work queues: group g holds item indices
// qitems[qrange[g].x .. qrange[g].y); qhead[g] is its cursor (zero before the launch).
// xcd_local: workgroups serve the group of the XCD they run on and frame barriers use
// XCD-local coherence; otherwise there is one group and agent-scope barriers.
// abort_flag: zero before the launch; raised by a workgroup whose barrier wait timed out
// so that every other wait ends at once.  budget = iterations per frame in this launch.
// Launch kinds of the fused kernel, each its own instantiation: frames gathering straight
// from memory, frames staging gather windows in LDS, one-workgroup frames with the whole
// solve in LDS.
// direct-fd: direct frames whose H pass forms the direction inside its gathers (batches
// whose direct frames all have P <= kFusedDirMaxPaths)
// windowed: frames tiled into strips whose gathers stream source rows through an LDS ring
constexpr int kKindDirect = 0, kKindStaged = 1, kKindResident = 2, kKindDirectFD = 3,
              kKindWindowed = 4, kKindLds = 5, kKinds = 6;
#ifndef OTFS_FUSED_DIR_MAX_PATHS
#define OTFS_FUSED_DIR_MAX_PATHS 8
#endif
constexpr int kFusedDirMaxPaths = OTFS_FUSED_DIR_MAX_PATHS;
// frames of at least this many elements stream t (see FrameDev::stream_t)
constexpr int64_t kStreamTElems = 131072;
hipError_t launch_cg_fused(int kind, int sd, const FrameDev* frames, const WorkItem* items,
                           const int32_t* qitems, const int2* qrange, unsigned* qhead, int ngroups,
                           int grid, int budget, Bases bases, bool xcd_local, unsigned* abort_flag,
                           int lds_bytes, int64_t wait_us, hipStream_t s);
// Workgroups of the fused kernel of a launch kind that fit on one CU at once (occupancy)
// with lds_bytes of dynamic LDS.
int fused_blocks_per_cu(int kind, int sd, int lds_bytes);
// FP64 true-residual refresh of the frames whose state is marked `refresh`, over all
// nitems work items (one workgroup each): two launches, u = y - H x, then
// c = H^H u - lam x with the FP64 partial norms in part_d.  Also clears every frame's
// barrier and neighbour counters and the nq queue cursors for the next fused launch.
// lds_bytes: dynamic LDS for the windows of frames with the windowed paired geometry (the
// largest window of the windowed kind's launch; 0 = every frame gathers from memory).
// nxcd: XCDs over which the device dispatches workgroups round robin (1: no such layout);
// the blocks of one XCD then take consecutive items, so a frame's tiles share its L2.
hipError_t launch_refresh(const FrameDev* frames, const WorkItem* items, int nitems, Bases bases,
                          unsigned* qhead, int nq, int lds_bytes, int nxcd, hipStream_t s);

// Static scratch of the entry point that allocates nothing: kNoAllocBytes per device.
// *ptr = its device address on `device`, which must be the current device (found once per
// device with hipGetSymbolAddress, then cached).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void** ptr);

// out[b] = XCC id of workgroup b, for b < nblocks.
hipError_t launch_xcc_probe(int* out, int nblocks, hipStream_t s);

// Plain (unfused, one frame per launch sequence) form of one frame.
hipError_t launch_plain_frame(const FrameDev* frames_dev, int frame, const WorkItem* items_dev,
                              int item_begin, int ntiles, int max_iters, Bases bases,
                              hipStream_t s);

// Paths of every frame from its received pilot frame (one workgroup per frame): the
// estimate Y (Hadamard) E_twist of Eq. heff_hadamard, the bins with |h|^2 > theta^2 (FP32
// test) in vector order, the first F.pcap of them made the frame's paths on the device
// (path table, P, shift ranges, FP32 and, where present, FP64 delay-ramp tables).
// ypilot: batch-wide complex64 pilot frames (frame at + off).  npaths[f] (nullable)
// receives the number of bins above the threshold.
hipError_t launch_pilot_paths(FrameDev* frames, int nframes, const float2* ypilot, float theta,
                              int32_t* npaths, hipStream_t s);

// Bit errors of the decisions sym against the transmitted indices tx (batch buffers), per
// frame, added to errs[frame] (cleared first when clear); frames without QAM are skipped.
hipError_t launch_bit_errors(const FrameDev* frames, const WorkItem* items, int nitems,
                             const uint8_t* sym, const uint8_t* tx, unsigned long long* errs,
                             int nframes, bool clear, hipStream_t s);
// Decisions and bit errors of the current estimates (x with a running frame's pending
// update applied) into B.sym and errs[frame].
hipError_t launch_trace_errors(const FrameDev* frames, const WorkItem* items, int nitems, Bases B,
                               const uint8_t* tx, unsigned long long* errs, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s);

// One piece of a gather copy: `bytes` bytes from device address src to byte offset dst of
// the destination buffer (src and dst 16-byte aligned).
struct CopySeg {
  const unsigned char* src;
  uint64_t dst;
  uint64_t bytes;
};
// Copy nseg segments (device array segs) into dst, one workgroup per segment.
hipError_t launch_gather_segments(const CopySeg* segs, int nseg, unsigned char* dst,
                                  hipStream_t s);

// Discrete Zak transform (inverse = false, Eq. zak) or its inverse (Eq. iZak) of nframes
// frames of M x N complex64 samples (dzt.hip): batched GEMM on MFMA.  in and out distinct.
hipError_t launch_dzt(int M, int N, int nframes, bool inverse, const float2* in, float2* out,
                      hipStream_t s);
constexpr int kDztMaxN = 8192;   // twiddle table of N complex64 values in LDS (64 KiB)

// Build the stored D table of every frame (sd = kDBf16 or kDC64).
hipError_t launch_build_d(int sd, const FrameDev* frames, const WorkItem* items, int nitems,
                          hipStream_t s);

}  // namespace otfs
