// Serving: continuous batching of LMMSE-CG frames that arrive over time.
//
// A scheduler thread owns the device side.  Frames wait in a FIFO queue until their state
// fits the caller's pool (the HBM admission budget); an admitted frame gets one slot of
// the pool holding its vectors, tables and CG state.  Each step runs `step_iters` CG
// iterations of every admitted frame in one launch of the fused kernel; the frames'
// state stays on the device between steps, frames that finish are copied out and leave,
// and frames that arrived meanwhile are admitted before the next step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "otfs_internal.h"
#include "plan_internal.h"

namespace otfs {
namespace {

using Clock = std::chrono::steady_clock;

#ifndef OTFS_SERVE_TILE
#define OTFS_SERVE_TILE 32768
#endif
constexpr int kServeTileElems = OTFS_SERVE_TILE;   // frame-local tiling rule (independent of the mix)
}  // namespace
int serve_tile_elems() { return kServeTileElems; }
namespace {
constexpr int kMaxActive = 2048;        // frames admitted at once
constexpr int kMaxItems = 65536;        // tiles of the admitted frames
constexpr size_t kAlign = 256;
constexpr int kDryRunCap = 512;         // resident workgroups assumed by a dry run

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing free blocks.
class PoolAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

// Byte offsets inside one frame's slot.  The inputs (y, tables, paths, initial state) come
// first, in [0, in_bytes): the submitting thread writes them into one page-locked host
// buffer of the same layout, and admission is a single copy of that buffer.
struct SlotLayout {
  size_t y, rtab, wtab, rtab64, wtab64, paths, st, in_bytes, x, c, p0, p1, t, a, u, part_pa,
      part_cc, part_d, bar, prog, sym, total;
};

SlotLayout slot_layout(const HostFrame& f, int tiles, bool refresh) {
  SlotLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = align_up(o + b);
    return at;
  };
  const size_t E = (size_t)f.M * f.N;
  L.y = take(E * 8);
  L.rtab = take((size_t)f.P * f.M * 8);
  L.wtab = take((size_t)f.N * 8);
  L.rtab64 = refresh ? take((size_t)f.P * f.M * 16) : 0;
  L.wtab64 = refresh ? take((size_t)f.N * 16) : 0;
  L.paths = take((size_t)f.P * 8);
  L.st = take(sizeof(FrameState));
  L.in_bytes = o;
  L.x = take(E * 8);
  L.c = take(E * 8);
  L.p0 = take(E * 8);
  L.p1 = take(E * 8);
  L.t = take(E * 8);
  L.a = take(E * 8);
  L.u = refresh ? take(E * 8) : 0;
  L.part_pa = take((size_t)tiles * 4);
  L.part_cc = take((size_t)tiles * 4);
  L.part_d = take((size_t)tiles * 8);
  L.bar = take(4);
  L.prog = take((size_t)tiles * 4);
  L.sym = take(E);
  L.total = o;
  return L;
}

// Control region at the start of the pool: step descriptors.
struct CtrlLayout {
  size_t frames, items, qitems, qrange, qhead, abort, stats, probe, segs, mirror, results, total;
};
// Device staging of finished frames' results (x-hat and decisions), gathered by a kernel
// and copied to the host in one piece per chunk of this size.
constexpr size_t kResultStage = (size_t)32 << 20;
CtrlLayout ctrl_layout() {
  CtrlLayout C{};
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = align_up(o + b);
    return at;
  };
  C.frames = take(kMaxActive * sizeof(FrameDev));
  C.items = take(kMaxItems * sizeof(WorkItem));
  C.qitems = take(kMaxItems * sizeof(int32_t));
  C.qrange = take(kKinds * kMaxGroups * sizeof(int2));
  C.qhead = take(kKinds * kMaxGroups * sizeof(unsigned));
  C.abort = take(sizeof(unsigned));
  C.stats = take(kMaxActive * sizeof(otfs_frame_stats));
  C.probe = take(kProbeBlocks * sizeof(int));
  C.segs = take(2 * kMaxActive * sizeof(CopySeg));
  C.mirror = o;   // the host mirror holds everything before the result staging
  C.results = take(kResultStage);
  C.total = o;
  return C;
}

// Host staging buffers of a server, kept per size and reused (frame shapes repeat):
// page-locked memory on a device, so that the copies to and from the pool are direct DMA
// instead of going through the driver's pageable staging; plain memory for the dry run,
// or when page-locking fails.
class HostPool {
 public:
  explicit HostPool(bool pinned) : pinned_(pinned) {}
  HostPool(const HostPool&) = delete;
  HostPool& operator=(const HostPool&) = delete;
  ~HostPool() {
    for (auto& kv : free_)
      for (void* p : kv.second) {
        if (locked_.count(p)) (void)hipHostFree(p);
        else std::free(p);
      }
  }
  // Buffers are kept per size class (eight classes per power of two, at most 12.5 % over the
  // request), so frames whose shapes or path counts differ a little reuse each other's.
  static size_t size_class(size_t n) {
    if (n <= 4096) return 4096;
    int b = 63 - __builtin_clzll((unsigned long long)n);   // 2^b <= n
    const size_t step = (size_t)1 << (b - 3);
    return (n + step - 1) / step * step;
  }
  void* get(size_t n) {
    n = size_class(n);
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = free_.find(n);
      if (it != free_.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    if (pinned_) {
      if (hipHostMalloc(&p, n, hipHostMallocPortable) == hipSuccess && p) {
        std::lock_guard<std::mutex> g(mu_);
        locked_.insert(p);
        return p;
      }
      (void)hipGetLastError();   // do not leave the failure for a later status check
    }
    return std::malloc(n);
  }
  void put(void* p, size_t n) {
    n = size_class(n);
    std::lock_guard<std::mutex> g(mu_);
    free_[n].push_back(p);
  }

 private:
  bool pinned_;
  std::mutex mu_;
  std::unordered_map<size_t, std::vector<void*>> free_;
  std::unordered_set<void*> locked_;
};

// One buffer from a HostPool, returned to it when reset or destroyed.
struct HostBuf {
  std::shared_ptr<HostPool> pool;
  void* p = nullptr;
  size_t n = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() { reset(); }
  void reset() {
    if (p) pool->put(p, n);
    p = nullptr;
    n = 0;
  }
  bool take(const std::shared_ptr<HostPool>& pl, size_t bytes) {
    reset();
    pool = pl;
    p = pl->get(bytes);
    n = p ? bytes : 0;
    return p != nullptr;
  }
  bool empty() const { return p == nullptr; }
};

struct Request {
  uint64_t ticket = 0;
  HostFrame hf;
  HostBuf in;                    // the slot's input region: y, tables, paths, initial state
  Clock::time_point t_submit, t_done;
  int state = 0;   // 0 queued, 1 admitted, 2 done
  // slot
  size_t slot_off = 0;
  SlotLayout L{};
  int tiles = 1;
  std::vector<WorkItem> items;   // frame-local tiles (frame index patched per step)
  FrameDev dev{};
  FrameDev geo{};                // staging geometry
  // `in` is filled at submission and stays alive until the frame is done, so the
  // admission copy needs no synchronisation
  // results
  // results: x-hat (complex64, M*N) at res_x and the decisions (u8, M*N, QAM frames) at
  // res_sym of a host buffer that the frames finished in the same chunk share
  std::shared_ptr<HostBuf> res;
  size_t res_x = 0, res_sym = 0;
  otfs_frame_stats stats{};
};

}  // namespace
}  // namespace otfs

using namespace otfs;

namespace otfs {
int serve_tile_elems();
}

struct otfs_server {
  int device = -1;
  bool dry = false;
  char* pool = nullptr;
  size_t pool_bytes = 0;
  otfs_cg_opts opts{};
  int step_iters = 10;
  CtrlLayout C{};
  PoolAlloc alloc;
  size_t slot_base = 0;   // first byte of the slot area (after the control region)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::shared_ptr<HostPool> hpool;
  std::vector<Request*> active;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool failed = false;
  std::string fail_msg;
  std::thread th;
  // device objects (scheduler thread)
  hipStream_t s = nullptr;
  XcdInfo xcd;
  int cus = 256;
  int cap = 0;              // workgroups of the fused kernel resident at once
  bool ready = false;       // scheduler_init finished
  int active_tiles = 0;
  // page-locked mirror of the control region: step descriptors are built here and copied
  // by DMA; the step's per-frame stats come back into it
  HostBuf stage;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;   // around a step's launches
  // counters
  uint64_t submitted = 0, completed = 0, steps = 0, peak = 0;
  uint64_t ns_admit = 0, ns_step = 0, ns_gpu = 0, ns_fetch = 0;   // scheduler time split
  // per-shape tile sizes (otfs_server_set_tiling); other shapes use serve_tile_elems()
  std::map<std::pair<int, int>, int> tile_of_shape;
  int tile_elems(const otfs::HostFrame& f) {
    std::lock_guard<std::mutex> g(mu);
    auto it = tile_of_shape.find({f.M, f.N});
    return it == tile_of_shape.end() ? otfs::serve_tile_elems() : it->second;
  }
};

namespace otfs {
namespace {

bool frame_fits_ever(otfs_server* S, const SlotLayout& L) {
  return L.total <= S->pool_bytes - S->slot_base;
}

// Host-side tables of a frame (FP64 phases, FP32 copies for the kernels), its path list
// and initial state, written into the request's input buffer at the slot's offsets; built
// on the submitting thread.
void build_tables(bool refresh, Request* r) {
  const HostFrame& f = r->hf;
  const SlotLayout& L = r->L;
  char* in = static_cast<char*>(r->in.p);
  std::vector<double2> r64, w64;
  for (int p = 0; p < f.P; ++p) delay_ramp(f, p, r64);
  wrap_factors(f, w64);
  int2* paths = reinterpret_cast<int2*>(in + L.paths);
  for (int p = 0; p < f.P; ++p) paths[p] = make_int2(f.tau[p], f.nu[p]);
  float2* r32 = reinterpret_cast<float2*>(in + L.rtab);
  float2* w32 = reinterpret_cast<float2*>(in + L.wtab);
  for (size_t i = 0; i < r64.size(); ++i) r32[i] = make_float2((float)r64[i].x, (float)r64[i].y);
  for (size_t i = 0; i < w64.size(); ++i) w32[i] = make_float2((float)w64[i].x, (float)w64[i].y);
  if (refresh) {
    std::memcpy(in + L.rtab64, r64.data(), r64.size() * sizeof(double2));
    std::memcpy(in + L.wtab64, w64.data(), w64.size() * sizeof(double2));
  }
  FrameState st0{};
  st0.status = OTFS_FRAME_RUNNING;
  std::memcpy(in + L.st, &st0, sizeof st0);
}

// Descriptor of an admitted frame (device pointers into its slot).
void build_frame_dev(otfs_server* S, Request* r) {
  const HostFrame& f = r->hf;
  char* base = S->pool + S->slot_base + r->slot_off;
  const SlotLayout& L = r->L;
  const bool refresh = S->opts.refresh_every > 0;
  FrameDev& d = r->dev;
  std::memset(&d, 0, sizeof d);
  d.y = base + L.y;
  d.x = reinterpret_cast<float2*>(base + L.x);
  d.c = reinterpret_cast<float2*>(base + L.c);
  d.p0 = reinterpret_cast<float2*>(base + L.p0);
  d.p1 = reinterpret_cast<float2*>(base + L.p1);
  d.t = reinterpret_cast<float2*>(base + L.t);
  d.a = reinterpret_cast<float2*>(base + L.a);
  d.u = refresh ? reinterpret_cast<float2*>(base + L.u) : nullptr;
  d.rtab = reinterpret_cast<const float2*>(base + L.rtab);
  d.wtab = reinterpret_cast<const float2*>(base + L.wtab);
  d.rtab64 = refresh ? reinterpret_cast<const double2*>(base + L.rtab64) : nullptr;
  d.wtab64 = refresh ? reinterpret_cast<const double2*>(base + L.wtab64) : nullptr;
  d.paths = reinterpret_cast<const int2*>(base + L.paths);
  d.part_pa = reinterpret_cast<float*>(base + L.part_pa);
  d.part_cc = reinterpret_cast<float*>(base + L.part_cc);
  d.part_d = reinterpret_cast<double*>(base + L.part_d);
  d.bar = reinterpret_cast<unsigned*>(base + L.bar);
  d.prog = reinterpret_cast<unsigned*>(base + L.prog);
  d.st = reinterpret_cast<FrameState*>(base + L.st);
  d.sym = f.qam > 0 ? reinterpret_cast<uint8_t*>(base + L.sym) : nullptr;
  frame_scalars(f, S->opts, r->tiles, r->geo, &d);
}

void set_failed(otfs_server* S, const std::string& msg) {
  std::lock_guard<std::mutex> g(S->mu);
  S->failed = true;
  S->fail_msg = msg;
  S->cv.notify_all();
}

// ---- GPU executor steps (scheduler thread) ----------------------------------------------
// Enqueue the copy of an admitted frame's inputs into its slot: one copy from page-locked
// memory (stream order puts it before the next step; the source lives in the request until
// it is done).
bool gpu_admit(otfs_server* S, Request* r) {
  build_frame_dev(S, r);
  char* base = S->pool + S->slot_base + r->slot_off;
  const hipError_t e = hipMemcpyAsync(base, r->in.p, r->L.in_bytes, hipMemcpyHostToDevice, S->s);
  if (e != hipSuccess) {
    set_failed(S, std::string("admission copy: ") + hipGetErrorString(e));
    return false;
  }
  return true;
}

bool gpu_step(otfs_server* S, std::vector<Request*>& act, std::vector<otfs_frame_stats>& out) {
  const int n = (int)act.size();
  const CtrlLayout& C = S->C;
  char* H = static_cast<char*>(S->stage.p);
  FrameDev* fd = reinterpret_cast<FrameDev*>(H + C.frames);
  WorkItem* items_h = reinterpret_cast<WorkItem*>(H + C.items);
  std::vector<HostFrame> frames(n);
  std::vector<int> tile_base(n), tiles(n);
  otfs_frame_stats* dstats = reinterpret_cast<otfs_frame_stats*>(S->pool + C.stats);
  int nitems = 0;
  for (int i = 0; i < n; ++i) {
    Request* r = act[i];
    fd[i] = r->dev;
    fd[i].stats = dstats + i;
    fd[i].index = i;
    frames[i] = r->hf;
    tile_base[i] = nitems;
    tiles[i] = r->tiles;
    if (nitems + (int)r->items.size() > kMaxItems) {
      set_failed(S, "too many tiles in one step");
      return false;
    }
    for (WorkItem w : r->items) {
      w.frame = i;
      items_h[nitems++] = w;
    }
  }
  std::vector<int32_t> qitems;
  std::vector<int2> qrange;
  std::vector<FrameDev> geo(n);
  for (int i = 0; i < n; ++i) geo[i] = act[i]->geo;
  std::vector<KindLaunch> launches;
  if (plan_launches(frames, geo, tile_base, tiles, kDNone, S->opts.refresh_every > 0,
                    (S->opts.flags & OTFS_SPLIT_DIRECTION) != 0, S->cus, 0, S->xcd, (S->opts.flags & OTFS_AGENT_BARRIER) != 0, qitems, qrange,
                    launches) != OTFS_OK) {
    set_failed(S, otfs_last_error());
    return false;
  }
  std::memcpy(H + C.qitems, qitems.data(), qitems.size() * sizeof(int32_t));
  std::memcpy(H + C.qrange, qrange.data(), qrange.size() * sizeof(int2));
  char* P = S->pool;
  hipError_t e = hipSuccess;
  auto up = [&](size_t off, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(P + off, H + off, bytes, hipMemcpyHostToDevice, S->s);
  };
  up(C.frames, (size_t)n * sizeof(FrameDev));
  up(C.items, (size_t)nitems * sizeof(WorkItem));
  up(C.qitems, qitems.size() * sizeof(int32_t));
  up(C.qrange, qrange.size() * sizeof(int2));
  const FrameDev* dframes = reinterpret_cast<const FrameDev*>(P + C.frames);
  unsigned* qhead = reinterpret_cast<unsigned*>(P + C.qhead);
  unsigned* abort_flag = reinterpret_cast<unsigned*>(P + C.abort);
  if (e == hipSuccess) e = hipEventRecord(S->ev_begin, S->s);
  if (e == hipSuccess)
    e = launch_step_reset(dframes, n, abort_flag, qhead, kKinds * kMaxGroups, S->s);
  Bases B{nullptr, nullptr, nullptr, nullptr};
  for (const KindLaunch& L : launches) {
    if (e != hipSuccess) break;
    e = launch_cg_fused(L.kind, kDNone, dframes, reinterpret_cast<const WorkItem*>(P + C.items),
                        reinterpret_cast<const int32_t*>(P + C.qitems),
                        reinterpret_cast<const int2*>(P + C.qrange) + L.qbase, qhead + L.qbase,
                        L.ngroups, L.grid, S->step_iters, B, L.xcd_local, abort_flag,
                        L.lds_bytes, -1, S->s);
  }
  // frames that reached a refresh point in this step get their FP64 true residual before
  // the next step resumes them
  if (e == hipSuccess && S->opts.refresh_every > 0)
    e = launch_refresh(dframes, reinterpret_cast<const WorkItem*>(P + C.items), nitems,
                       B, qhead, kKinds * kMaxGroups, refresh_lds_bytes(launches),
                       S->xcd.round_robin ? S->xcd.nxcd : 1, S->s);
  if (e == hipSuccess) e = hipEventRecord(S->ev_end, S->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(H + C.stats, dstats, (size_t)n * sizeof(otfs_frame_stats),
                       hipMemcpyDeviceToHost, S->s);
  if (e == hipSuccess) e = hipStreamSynchronize(S->s);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, S->ev_begin, S->ev_end);
  if (e != hipSuccess) {
    set_failed(S, std::string("serving step: ") + hipGetErrorString(e));
    return false;
  }
  out.resize(n);
  std::memcpy(out.data(), H + C.stats, (size_t)n * sizeof(otfs_frame_stats));
  S->ns_gpu += (uint64_t)((double)ms * 1e6);
  return true;
}

// Results of the frames finished in a step.  Chunk by chunk (up to kResultStage bytes), a
// kernel gathers the frames' x-hat and decisions from their slots into the staging region
// and one copy brings the chunk to a page-locked host buffer that those frames share; a
// frame too large for the staging region is copied from its slot directly.
bool gpu_fetch(otfs_server* S, const std::vector<Request*>& done) {
  const CtrlLayout& C = S->C;
  char* H = static_cast<char*>(S->stage.p);
  CopySeg* segs_h = reinterpret_cast<CopySeg*>(H + C.segs);
  const CopySeg* segs_d = reinterpret_cast<const CopySeg*>(S->pool + C.segs);
  unsigned char* stage_d = reinterpret_cast<unsigned char*>(S->pool + C.results);
  hipError_t e = hipSuccess;
  auto result_bytes = [](const Request* r, size_t* xo, size_t* so) {
    const size_t E = (size_t)r->hf.M * r->hf.N;
    *xo = 0;
    *so = align_up(E * sizeof(float2));
    return align_up(*so + (r->hf.qam > 0 ? E : 0));
  };
  size_t i = 0;
  while (e == hipSuccess && i < done.size()) {
    size_t xo, so;
    const size_t b0 = result_bytes(done[i], &xo, &so);
    auto buf = std::make_shared<HostBuf>();
    if (b0 > kResultStage) {   // alone, straight from its slot
      Request* r = done[i];
      const size_t E = (size_t)r->hf.M * r->hf.N;
      if (!buf->take(S->hpool, b0)) {
        set_failed(S, "result copy: out of host memory");
        return false;
      }
      char* base = S->pool + S->slot_base + r->slot_off;
      char* hb = static_cast<char*>(buf->p);
      e = hipMemcpyAsync(hb + xo, base + r->L.x, E * sizeof(float2), hipMemcpyDeviceToHost, S->s);
      if (e == hipSuccess && r->hf.qam > 0)
        e = hipMemcpyAsync(hb + so, base + r->L.sym, E, hipMemcpyDeviceToHost, S->s);
      if (e == hipSuccess) e = hipStreamSynchronize(S->s);
      r->res = buf;
      r->res_x = xo;
      r->res_sym = so;
      ++i;
      continue;
    }
    // frames [i, j) fill this chunk
    size_t used = 0;
    int nseg = 0;
    size_t j = i;
    for (; j < done.size(); ++j) {
      Request* r = done[j];
      const size_t b = result_bytes(r, &xo, &so);
      if (b > kResultStage || used + b > kResultStage) break;
      const size_t E = (size_t)r->hf.M * r->hf.N;
      const unsigned char* base =
          reinterpret_cast<const unsigned char*>(S->pool + S->slot_base + r->slot_off);
      segs_h[nseg++] = CopySeg{base + r->L.x, used + xo, E * sizeof(float2)};
      if (r->hf.qam > 0) segs_h[nseg++] = CopySeg{base + r->L.sym, used + so, E};
      r->res_x = used + xo;
      r->res_sym = used + so;
      used += b;
    }
    if (!buf->take(S->hpool, used)) {
      set_failed(S, "result copy: out of host memory");
      return false;
    }
    e = hipMemcpyAsync(S->pool + C.segs, segs_h, (size_t)nseg * sizeof(CopySeg),
                       hipMemcpyHostToDevice, S->s);
    if (e == hipSuccess) e = launch_gather_segments(segs_d, nseg, stage_d, S->s);
    if (e == hipSuccess) e = hipMemcpyAsync(buf->p, stage_d, used, hipMemcpyDeviceToHost, S->s);
    // the segment list in the host mirror is rewritten by the next chunk: wait here
    if (e == hipSuccess) e = hipStreamSynchronize(S->s);
    for (size_t k = i; k < j; ++k) done[k]->res = buf;
    i = j;
  }
  if (e != hipSuccess) {
    set_failed(S, std::string("result copy: ") + hipGetErrorString(e));
    return false;
  }
  return true;
}

// ---- scheduler ---------------------------------------------------------------------------
// Device set-up of the scheduler thread: stream, XCD layout, resident workgroups.
bool scheduler_init(otfs_server* S) {
  if (S->dry) {
    S->cap = kDryRunCap;
    return true;
  }
  hipError_t e = hipSetDevice(S->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking);
  if (e != hipSuccess) {
    set_failed(S, std::string("server stream: ") + hipGetErrorString(e));
    return false;
  }
  if (probe_xcds(S->device, S->pool + S->C.probe, S->s, &S->xcd) != OTFS_OK) {
    set_failed(S, std::string("XCC probe: ") + otfs_last_error());
    return false;
  }
  if (!S->stage.take(S->hpool, S->C.mirror)) {
    set_failed(S, "no host memory for the step descriptors");
    return false;
  }
  e = hipEventCreate(&S->ev_begin);
  if (e == hipSuccess) e = hipEventCreate(&S->ev_end);
  if (e != hipSuccess) {
    set_failed(S, std::string("server events: ") + hipGetErrorString(e));
    return false;
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, S->device) == hipSuccess && v > 0)
    S->cus = v;
  // the tile cap of a frame: workgroups of the direct kind resident at once
  S->cap = std::max(1, fused_blocks_per_cu(kKindDirect, kDNone, 0)) * S->cus;
  return true;
}

void scheduler(otfs_server* S) {
  const bool ok = scheduler_init(S);
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->ready = true;
  }
  S->cv.notify_all();
  if (!ok) return;
  std::vector<otfs_frame_stats> st;
  for (;;) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || S->failed || !S->queue.empty() || !S->active.empty(); });
      if (S->stop || S->failed) return;
      // admission: arrival order, while the head fits
      while (!S->queue.empty() && (int)S->active.size() + (int)admitted.size() < kMaxActive) {
        Request* r = S->queue.front();
        if (S->active_tiles + r->tiles > kMaxItems) break;
        size_t off = 0;
        if (!S->alloc.alloc(r->L.total, &off)) break;
        r->slot_off = off;
        r->state = 1;
        S->active_tiles += r->tiles;
        S->queue.pop_front();
        admitted.push_back(r);
      }
      S->peak = std::max<uint64_t>(S->peak, S->alloc.used());
    }
    const auto t_admit = Clock::now();
    for (Request* r : admitted) {
      if (!S->dry && !gpu_admit(S, r)) return;
    }
    const auto t_step = Clock::now();
    std::vector<Request*> act;
    {
      std::lock_guard<std::mutex> g(S->mu);
      for (Request* r : admitted) S->active.push_back(r);
      act = S->active;
    }
    if (act.empty()) continue;
    st.clear();
    if (S->dry) {
      // dry run: every frame finishes after ceil(max_iters / step_iters) steps
      st.resize(act.size());
      for (size_t i = 0; i < act.size(); ++i) {
        Request* r = act[i];
        r->stats.iters = std::min(S->opts.max_iters, r->stats.iters + S->step_iters);
        st[i] = otfs_frame_stats{r->stats.iters, 0.f,
                                 r->stats.iters >= S->opts.max_iters ? OTFS_FRAME_DRYRUN
                                                                     : OTFS_FRAME_RUNNING,
                                 r->tiles};
      }
    } else if (!gpu_step(S, act, st)) {
      return;
    }
    const auto t_fetch = Clock::now();
    std::vector<Request*> done;
    for (size_t i = 0; i < act.size(); ++i)
      if (st[i].status != OTFS_FRAME_RUNNING) {
        act[i]->stats = st[i];
        done.push_back(act[i]);
      }
    if (S->dry) {
      for (Request* r : done) {
        const size_t E = (size_t)r->hf.M * r->hf.N;
        auto buf = std::make_shared<HostBuf>();
        const size_t so = align_up(E * sizeof(float2));
        const size_t b = so + (r->hf.qam > 0 ? E : 0);
        if (buf->take(S->hpool, b)) std::memset(buf->p, 0, b);
        r->res = buf;
        r->res_x = 0;
        r->res_sym = so;
      }
    } else if (!gpu_fetch(S, done)) {
      return;
    }
    {
      std::lock_guard<std::mutex> g(S->mu);
      const auto now = Clock::now();
      auto ns = [](Clock::duration d) {
        return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(d).count();
      };
      S->ns_admit += ns(t_step - t_admit);
      S->ns_step += ns(t_fetch - t_step);
      S->ns_fetch += ns(now - t_fetch);
      for (Request* r : done) {
        r->t_done = now;
        r->state = 2;
        r->in.reset();   // its admission copy finished at an earlier step's synchronisation
        S->alloc.release(r->slot_off, r->L.total);
        S->active_tiles -= r->tiles;
        S->active.erase(std::find(S->active.begin(), S->active.end(), r));
        ++S->completed;
      }
      ++S->steps;
    }
    S->cv.notify_all();
  }
}

}  // namespace
}  // namespace otfs

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" otfs_status otfs_server_create(int device, void* pool_dev, size_t pool_bytes,
                                          const otfs_cg_opts* opts, int32_t step_iters,
                                          otfs_server_t** out) {
  if (!out) return fail(OTFS_E_INVAL, "out must be non-null");
  *out = nullptr;
  if (device < -1) return fail(OTFS_E_INVAL, "device must be >= 0, or -1 for a dry run");
  if (step_iters < 1) return fail(OTFS_E_INVAL, "step_iters must be >= 1");
  otfs_cg_opts o{};
  otfs_status st = validate_opts(opts, &o);
  if (st != OTFS_OK) return st;
  if (o.flags & (OTFS_D_STORED_BF16 | OTFS_D_STORED_C64 | OTFS_Y_BF16))
    return fail(OTFS_E_UNSUPPORTED, "the stored-D and bf16 flags are not supported by the server");
  if (device >= 0) {
    if (!pool_dev) return fail(OTFS_E_INVAL, "pool_dev is null");
    if ((reinterpret_cast<uintptr_t>(pool_dev) & 255u) != 0)
      return fail(OTFS_E_INVAL, "pool_dev must be 256-byte aligned");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev)
      return fail(OTFS_E_INVAL, "no device %d", device);
  }
  auto S = std::make_unique<otfs_server>();
  S->device = device;
  S->dry = device < 0;
  S->hpool = std::make_shared<HostPool>(!S->dry);
  S->pool = static_cast<char*>(pool_dev);
  S->pool_bytes = pool_bytes;
  S->opts = o;
  S->step_iters = step_iters;
  S->C = ctrl_layout();
  S->slot_base = S->C.total;
  if (pool_bytes <= S->slot_base)
    return fail(OTFS_E_BUDGET, "pool of %zu bytes is smaller than the %zu-byte control region",
                pool_bytes, S->slot_base);
  S->alloc.reset(pool_bytes - S->slot_base);
  otfs_server* raw = S.release();
  try {
    raw->th = std::thread(scheduler, raw);
  } catch (...) {
    delete raw;
    return fail(OTFS_E_NOMEM, "could not start the scheduler thread");
  }
  std::string err;
  {
    std::unique_lock<std::mutex> lk(raw->mu);
    raw->cv.wait(lk, [&] { return raw->ready; });
    if (raw->failed) err = raw->fail_msg;
  }
  if (!err.empty()) {
    otfs_server_free(raw);
    return fail(OTFS_E_DEVICE, "server start: %s", err.c_str());
  }
  *out = raw;
  return OTFS_OK;
}

namespace otfs {
namespace {
// A request for one frame: validation, tiling, slot layout, its inputs copied into a
// page-locked buffer and its tables built (the submitting thread's share of the work).
otfs_status make_request(otfs_server* S, const otfs_frame_desc& frame, const void* y_host,
                         std::unique_ptr<Request>* out) {
  auto r = std::make_unique<Request>();
  otfs_status st = validate_frame(frame, 0, &r->hf);
  if (st != OTFS_OK) return st;
  const size_t E = (size_t)frame.M * frame.N;
  std::vector<WorkItem> items;
  std::vector<int> tb, tl;
  make_tiles(std::vector<HostFrame>{r->hf}, S->tile_elems(r->hf), items, tb, tl);
  r->tiles = tl[0];
  r->items = items;
  int band = 1;
  for (const WorkItem& w : items) band = std::max(band, w.l_end - w.l_begin);
  lds_geometry(r->hf, r->tiles, band, S->opts, kDefaultStageBytes, &r->geo);
  if (r->tiles > S->cap || r->tiles > kMaxItems)
    return fail(OTFS_E_UNSUPPORTED, "frame needs %d cooperating workgroups, %d fit", r->tiles,
                std::min(S->cap, kMaxItems));
  r->L = slot_layout(r->hf, r->tiles, S->opts.refresh_every > 0);
  if (!frame_fits_ever(S, r->L))
    return fail(OTFS_E_BUDGET, "frame state needs %zu bytes, the pool has %zu for frames",
                r->L.total, S->pool_bytes - S->slot_base);
  if (!r->in.take(S->hpool, r->L.in_bytes))
    return fail(OTFS_E_NOMEM, "no host memory for the frame's inputs");
  std::memcpy(static_cast<char*>(r->in.p) + r->L.y, y_host, E * sizeof(float2));
  build_tables(S->opts.refresh_every > 0, r.get());
  *out = std::move(r);
  return OTFS_OK;
}

// Queue requests in order (S->mu held): tickets, submit times, the scheduler's queue.
void enqueue_locked(otfs_server* S, std::vector<std::unique_ptr<Request>>& rs, uint64_t* tickets) {
  const auto now = Clock::now();
  for (size_t i = 0; i < rs.size(); ++i) {
    Request* raw = rs[i].get();
    raw->t_submit = now;
    raw->ticket = S->next_ticket++;
    tickets[i] = raw->ticket;
    S->reqs.emplace(raw->ticket, std::move(rs[i]));
    S->queue.push_back(raw);
    ++S->submitted;
  }
}
}  // namespace
}  // namespace otfs

extern "C" otfs_status otfs_submit(otfs_server_t* S, const otfs_frame_desc* frame,
                                   const void* y_host, uint64_t* ticket) {
  return otfs_submit_many(S, frame, 1, &y_host, ticket);
}

extern "C" otfs_status otfs_submit_many(otfs_server_t* S, const otfs_frame_desc* frames,
                                        int32_t n, const void* const* y_host,
                                        uint64_t* tickets) {
  if (!S || n < 0 || (n > 0 && (!frames || !y_host || !tickets)))
    return fail(OTFS_E_INVAL, "null argument or negative count");
  std::vector<std::unique_ptr<Request>> rs((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    if (!y_host[i]) return fail(OTFS_E_INVAL, "y_host[%d] is null", i);
    const otfs_status st = make_request(S, frames[i], y_host[i], &rs[i]);
    if (st != OTFS_OK) return st;   // nothing queued
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->failed) return fail(OTFS_E_DEVICE, "server failed: %s", S->fail_msg.c_str());
    enqueue_locked(S, rs, tickets);
  }
  S->cv.notify_all();
  return OTFS_OK;
}

extern "C" otfs_status otfs_server_set_tiling(otfs_server_t* S, int32_t M, int32_t N,
                                              int32_t tile_elems) {
  if (!S) return fail(OTFS_E_INVAL, "server is null");
  if (M < 1 || N < 1 || tile_elems < 0)
    return fail(OTFS_E_INVAL, "need M, N >= 1 and tile_elems >= 0");
  std::lock_guard<std::mutex> g(S->mu);
  if (tile_elems == 0)
    S->tile_of_shape.erase({M, N});
  else
    S->tile_of_shape[{M, N}] = tile_elems;
  return OTFS_OK;
}

extern "C" otfs_status otfs_server_frame_bytes(otfs_server_t* S, const otfs_frame_desc* frame,
                                               size_t* frame_bytes, size_t* control_bytes) {
  if (!S || !frame) return fail(OTFS_E_INVAL, "null argument");
  HostFrame hf;
  otfs_status st = validate_frame(*frame, 0, &hf);
  if (st != OTFS_OK) return st;
  std::vector<WorkItem> items;
  std::vector<int> tb, tl;
  make_tiles(std::vector<HostFrame>{hf}, S->tile_elems(hf), items, tb, tl);
  if (frame_bytes) *frame_bytes = slot_layout(hf, tl[0], S->opts.refresh_every > 0).total;
  if (control_bytes) *control_bytes = S->slot_base;
  return OTFS_OK;
}

namespace otfs {
namespace {
// Copy a finished request's results out (no lock needed: the request is no longer shared).
void deliver(const Request& r, void* xhat_host, uint8_t* sym_host, otfs_frame_stats* stats,
             uint64_t* latency_ns) {
  const size_t E = (size_t)r.hf.M * r.hf.N;
  if (r.res && !r.res->empty()) {
    const char* hb = static_cast<const char*>(r.res->p);
    if (xhat_host) std::memcpy(xhat_host, hb + r.res_x, E * sizeof(float2));
    if (sym_host && r.hf.qam > 0) std::memcpy(sym_host, hb + r.res_sym, E);
  }
  if (stats) *stats = r.stats;
  if (latency_ns)
    *latency_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(r.t_done - r.t_submit).count();
}
}  // namespace
}  // namespace otfs

extern "C" otfs_status otfs_poll(otfs_server_t* S, uint64_t ticket, void* xhat_host,
                                 uint8_t* sym_host, otfs_frame_stats* stats,
                                 uint64_t* latency_ns) {
  if (!S) return fail(OTFS_E_INVAL, "server is null");
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(OTFS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != 2) {
      if (S->failed) return fail(OTFS_E_DEVICE, "server failed: %s", S->fail_msg.c_str());
      return OTFS_E_AGAIN;
    }
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  deliver(*r, xhat_host, sym_host, stats, latency_ns);
  return OTFS_OK;
}

extern "C" otfs_status otfs_poll_many(otfs_server_t* S, const uint64_t* tickets, int32_t n,
                                      void* const* xhat_host, uint8_t* const* sym_host,
                                      otfs_frame_stats* stats, uint64_t* latency_ns,
                                      int32_t* status, int32_t* ndone) {
  if (!S || n < 0 || (n > 0 && (!tickets || !status)))
    return fail(OTFS_E_INVAL, "null argument or negative count");
  std::vector<std::pair<int32_t, std::unique_ptr<Request>>> got;
  {
    std::lock_guard<std::mutex> g(S->mu);
    for (int32_t i = 0; i < n; ++i) {
      auto it = S->reqs.find(tickets[i]);
      if (it == S->reqs.end()) {
        status[i] = OTFS_E_NOTFOUND;
      } else if (it->second->state != 2) {
        status[i] = S->failed ? OTFS_E_DEVICE : OTFS_E_AGAIN;
      } else {
        status[i] = OTFS_OK;
        got.emplace_back(i, std::move(it->second));
        S->reqs.erase(it);
      }
    }
  }
  for (auto& gr : got) {
    const int32_t i = gr.first;
    deliver(*gr.second, xhat_host ? xhat_host[i] : nullptr, sym_host ? sym_host[i] : nullptr,
            stats ? stats + i : nullptr, latency_ns ? latency_ns + i : nullptr);
  }
  if (ndone) *ndone = (int32_t)got.size();
  return OTFS_OK;
}

extern "C" otfs_status otfs_server_stats(otfs_server_t* S, otfs_server_stats_t* out) {
  if (!S || !out) return fail(OTFS_E_INVAL, "null argument");
  std::lock_guard<std::mutex> g(S->mu);
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->steps = S->steps;
  out->queued = S->queue.size();
  out->active = S->active.size();
  out->pool_bytes_in_use = S->alloc.used();
  out->pool_bytes_peak = S->peak;
  out->ns_admit = S->ns_admit;
  out->ns_step = S->ns_step;
  out->ns_gpu = S->ns_gpu;
  out->ns_fetch = S->ns_fetch;
  if (S->failed) return fail(OTFS_E_DEVICE, "server failed: %s", S->fail_msg.c_str());
  return OTFS_OK;
}

extern "C" otfs_status otfs_server_free(otfs_server_t* S) {
  if (!S) return OTFS_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  if (S->s) {
    (void)hipStreamSynchronize(S->s);
    (void)hipStreamDestroy(S->s);
  }
  if (S->ev_begin) (void)hipEventDestroy(S->ev_begin);
  if (S->ev_end) (void)hipEventDestroy(S->ev_end);
  delete S;
  return OTFS_OK;
}
