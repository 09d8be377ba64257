// Host-side plan structures shared by plan.cpp and server.cpp.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "otfs_internal.h"

namespace otfs {

constexpr int kMaxPaths = 64;

// A validated frame descriptor, owned by the host.
struct HostFrame {
  int M = 0, N = 0, P = 0;
  float lam = 0.f;
  int qam = 0;
  std::vector<int> tau, nu;
  std::vector<float2> h;
  int64_t off = 0;   // element offset inside the batch
};

// Byte offsets of every region of a plan workspace.
struct Layout {
  size_t frames = 0, items = 0, qitems = 0, qrange = 0, qhead = 0, probe = 0;
  size_t rtab = 0, wtab = 0, rtab64 = 0, wtab64 = 0, paths = 0;
  size_t part_pa = 0, part_cc = 0, part_d = 0, bar = 0, prog = 0, st = 0, abort = 0;
  size_t c = 0, p0 = 0, p1 = 0, t = 0, a = 0, u = 0, dtab = 0;
  size_t total = 0;
};

struct GraphKey {
  const void* y;
  void* x;
  void* sym;
  void* stats;
  hipStream_t s;
  bool operator==(const GraphKey& o) const {
    return y == o.y && x == o.x && sym == o.sym && stats == o.stats && s == o.s;
  }
};

otfs_status fail(otfs_status st, const char* fmt, ...);
otfs_status hip_fail(hipError_t e, const char* what);
otfs_status validate_opts(const otfs_cg_opts* o, otfs_cg_opts* out);
otfs_status validate_frame(const otfs_frame_desc& f, int idx, HostFrame* out);
void delay_ramp(const HostFrame& f, int p, std::vector<double2>& out);
void wrap_factors(const HostFrame& f, std::vector<double2>& out);
void frame_scalars(const HostFrame& fr, const otfs_cg_opts& o, int tiles, const FrameDev& geo,
                   FrameDev* d);
int default_tile_elems(int64_t total_elems, int cus);
// Tiles of every frame: strips of winw[f] delay columns over all rows for windowed frames
// (winw non-null and winw[f] > 0), else bands of Doppler rows of about tile_elems elements.
void make_tiles(const std::vector<HostFrame>& frames, int tile_elems, std::vector<WorkItem>& items,
                std::vector<int>& tile_base, std::vector<int>& tiles,
                const std::vector<int>* winw = nullptr);
// Strip width a frame runs with in the windowed form for a requested strip width w and
// chunk of rc rows, or 0 when the frame does not meet the form's limits.
int window_width(const HostFrame& f, int w, int rc);
constexpr int kMaxLdsBytes = 160 * 1024;
// LDS of the windowed paired gathers' window (the workgroup's static LDS stays below 1 KiB)
constexpr int kLdsGatherBytes = kMaxLdsBytes - 1024;
int lds_pair_geometry(const HostFrame& f, int tiles, int budget_bytes, FrameDev* geo);
// Work queues of the fused kernel.  ngroups groups (one per XCD in XCD-local mode, else
// one); every frame's tiles go, consecutively, to one group; groups are balanced by work.
// per_group_cap: workgroups one group can hold resident.  Returns false if some frame has
// more tiles than that.
bool make_queues(const std::vector<HostFrame>& frames, const std::vector<int>& tile_base,
                 const std::vector<int>& tiles, int ngroups, int per_group_cap,
                 std::vector<int32_t>& qitems, std::vector<int2>& qrange, int* per_group_grid);
// XCD layout of a device, found once per device by a probe launch.
struct XcdInfo {
  int nxcd = 1;          // number of XCDs seen
  bool round_robin = false;  // workgroup b ran on XCD b % nxcd for every probed b
};
otfs_status probe_xcds(int device, void* scratch_dev, hipStream_t s, XcdInfo* out);
void retile(struct ::otfs_plan* pl);
// Staged-gather geometry of one frame whose widest tile has band_rows rows: fills
// skc/ssb (0 = direct gathers) and the shift ranges; returns the window size in elements.
int stage_geometry(const HostFrame& f, int band_rows, int budget_elems, FrameDev* d);
// LDS use of one frame within budget_bytes: the resident form for a one-tile frame whose
// vectors fit (no stored D, no refresh), else staged windows, else none.  Fills the
// geometry fields of *geo (resident, skc, ssb, shift ranges); returns the bytes it needs.
constexpr int kResidentVecs = 5;
int lds_geometry(const HostFrame& f, int tiles, int band_rows, const otfs_cg_opts& o,
                 int budget_bytes, FrameDev* geo);
constexpr int kProbeBlocks = 1024;

// One launch of the fused kernel: the frames of one kind with their work queues.  The
// queue ranges and cursors of launch kind k live at k * kMaxGroups.
struct KindLaunch {
  int kind = kKindDirect;
  int nframes = 0;          // frames of this kind
  int grid = 0;
  int ngroups = 1;
  bool xcd_local = false;
  int lds_bytes = 0;
  int qbase = 0;
};
// The refresh launches' LDS: the windowed paired kind's window bytes among `launches` (0
// when it has none).
int refresh_lds_bytes(const std::vector<KindLaunch>& launches);
int frame_kind(const FrameDev& geo);
// LDS a frame of this kind and geometry needs in its launch.
int frame_lds_bytes(const HostFrame& f, const FrameDev& geo);
// Work queues and launch shapes of every kind present among the frames (frames listed by
// index into tile_base / tiles; item indices are tile_base[f] + t).  cap_override > 0
// caps the workgroups of each launch.  Direct frames run the direct-fd kind when every
// one of them has P <= kFusedDirMaxPaths, neither stored nor refresh is on, and split_dir
// is false.  Fails if a frame has more tiles than can be resident at once.
otfs_status plan_launches(const std::vector<HostFrame>& frames, const std::vector<FrameDev>& geo,
                          const std::vector<int>& tile_base, const std::vector<int>& tiles,
                          int sd, bool refresh, bool split_dir, int cus, int cap_override,
                          const XcdInfo& xi, bool agent, std::vector<int32_t>& qitems,
                          std::vector<int2>& qrange, std::vector<KindLaunch>& out);

}  // namespace otfs

struct otfs_plan {
  std::vector<otfs::HostFrame> frames;
  otfs_cg_opts opts{};
  int64_t total_elems = 0;
  int max_paths = 0, cus = 256;
  int tile_elems = 0, max_grid_req = 0;
  int stage_bytes = otfs::kDefaultStageBytes;   // LDS budget for staged windows, 0 = off
  int64_t wait_us = -1;   // bound of the kernels' waits (-1: the default 20 s)
  int ref_xcds = 1;       // XCDs of round-robin dispatch (block order of the refresh)
  bool device_paths = false;   // the path tables were made on the device (from a pilot)
  int win_w_req = 0, win_rc_req = 0;   // windowed form (0: off)
  std::vector<int> winw;               // per frame: strip width of the windowed form, or 0
  // tiling (host) and schedule (chosen at bind)
  std::vector<otfs::WorkItem> items;
  std::vector<int> tile_base, tiles;
  std::vector<int32_t> qitems;
  std::vector<int2> qrange;
  std::vector<otfs::KindLaunch> launches;
  otfs::Layout L;
  // binding
  bool bound = false;
  int device = -1;
  void* ws = nullptr;
  otfs::FrameDev* d_frames = nullptr;
  otfs::WorkItem* d_items = nullptr;
  int32_t* d_qitems = nullptr;
  int2* d_qrange = nullptr;
  unsigned* d_qhead = nullptr;
  unsigned* d_abort = nullptr;
  // host copies of the uploaded tables (kept alive across the asynchronous copies)
  std::vector<float2> h_rtab, h_wtab;
  std::vector<double2> h_rtab64, h_wtab64;
  std::vector<int2> h_paths;
  std::vector<otfs::FrameDev> h_frames;
  // kernel timing
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  bool timed_pending = false;
  // captured launch sequence
  hipGraphExec_t gexec = nullptr;
  otfs::GraphKey gkey{};
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
};
