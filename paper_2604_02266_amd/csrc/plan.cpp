// Host side of libotfs: plan validation, coefficient tables, tiling and scheduling,
// workspace layout, and the batch entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <mutex>
#include <vector>

#include "otfs_internal.h"
#include "plan_internal.h"

namespace otfs {

// ---------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

otfs_status fail(otfs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

otfs_status hip_fail(hipError_t e, const char* what) {
  return fail(OTFS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------------------
// validation and tables
// ---------------------------------------------------------------------------------------
otfs_status validate_opts(const otfs_cg_opts* o, otfs_cg_opts* out) {
  otfs_cg_opts d{50, 1e-6f, 0, 0u};
  if (o) d = *o;
  if (d.max_iters < 1) return fail(OTFS_E_INVAL, "max_iters must be >= 1 (got %d)", d.max_iters);
  if (!(d.rel_tol >= 0.f) || !std::isfinite(d.rel_tol))
    return fail(OTFS_E_INVAL, "rel_tol must be finite and >= 0");
  if (d.refresh_every < 0) return fail(OTFS_E_INVAL, "refresh_every must be >= 0");
  const uint32_t known = OTFS_D_STORED_BF16 | OTFS_Y_BF16 | OTFS_USE_GRAPH | OTFS_TIME_KERNEL |
                         OTFS_LDS_GATHER |
                         OTFS_AGENT_BARRIER | OTFS_NO_LDS_RESIDENT | OTFS_SPLIT_DIRECTION |
                         OTFS_D_STORED_C64;
  if (d.flags & ~known) return fail(OTFS_E_INVAL, "unknown flag bits 0x%x", d.flags & ~known);
  if ((d.flags & OTFS_D_STORED_BF16) && (d.flags & OTFS_D_STORED_C64))
    return fail(OTFS_E_INVAL, "OTFS_D_STORED_BF16 and OTFS_D_STORED_C64 exclude each other");
  *out = d;
  return OTFS_OK;
}

otfs_status validate_frame(const otfs_frame_desc& f, int idx, HostFrame* out) {
  if (f.M < 1 || f.N < 1)
    return fail(OTFS_E_INVAL, "frame %d: M and N must be >= 1 (got %d x %d)", idx, f.M, f.N);
  const int64_t E = (int64_t)f.M * f.N;
  if (E > (int64_t(1) << 28))
    return fail(OTFS_E_INVAL, "frame %d: M*N = %lld exceeds 2^28", idx, (long long)E);
  if (f.P < 1 || f.P > kMaxPaths)
    return fail(OTFS_E_INVAL, "frame %d: P must be in [1, %d] (got %d)", idx, kMaxPaths, f.P);
  if (!f.h || !f.delay || !f.doppler)
    return fail(OTFS_E_INVAL, "frame %d: h, delay and doppler must be non-null", idx);
  if (!(f.noise_var >= 0.f) || !std::isfinite(f.noise_var))
    return fail(OTFS_E_INVAL, "frame %d: noise_var must be finite and >= 0", idx);
  if (!(f.qam == 0 || f.qam == 4 || f.qam == 16 || f.qam == 64 || f.qam == 256))
    return fail(OTFS_E_INVAL, "frame %d: qam must be 0, 4, 16, 64 or 256 (got %d)", idx, f.qam);
  HostFrame h;
  h.M = f.M;
  h.N = f.N;
  h.P = f.P;
  h.lam = f.noise_var;
  h.qam = f.qam;
  h.tau.resize(f.P);
  h.nu.resize(f.P);
  h.h.resize(f.P);
  for (int p = 0; p < f.P; ++p) {
    const int t = f.delay[p], v = f.doppler[p];
    if (t <= -f.M || t >= f.M)
      return fail(OTFS_E_INVAL, "frame %d path %d: need |delay| < M (delay %d, M %d)", idx, p, t, f.M);
    if (v <= -f.N || v >= f.N)
      return fail(OTFS_E_INVAL, "frame %d path %d: need |doppler| < N (doppler %d, N %d)", idx, p, v, f.N);
    const float re = f.h[2 * p], im = f.h[2 * p + 1];
    if (!std::isfinite(re) || !std::isfinite(im))
      return fail(OTFS_E_INVAL, "frame %d path %d: gain is not finite", idx, p);
    h.tau[p] = t;
    h.nu[p] = v;
    h.h[p] = {re, im};
  }
  // Paths in (Doppler, delay) order: consecutive paths of the gather loop then read the
  // same or neighbouring source rows, which the caches serve (the sum over paths is the
  // same; only its rounding order follows this order).
  std::vector<int> ord(h.P);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    return h.nu[a] != h.nu[b] ? h.nu[a] < h.nu[b] : h.tau[a] < h.tau[b];
  });
  HostFrame g = h;
  for (int p = 0; p < h.P; ++p) {
    g.tau[p] = h.tau[ord[p]];
    g.nu[p] = h.nu[ord[p]];
    g.h[p] = h.h[ord[p]];
  }
  *out = std::move(g);
  return OTFS_OK;
}

// R_p[k] = h_p e^{j 2 pi nu_p (k - tau_p) / (MN)} for k in [0, M).  With k = 32 kh + kl the
// phase splits into a block part nu_p (32 kh - tau_p) and an in-block part nu_p kl; each
// numerator is reduced modulo MN in exact integer arithmetic before its angle is formed in
// FP64, and R_p[k] is h_p times the product of the two unit phasors (about 2 sqrt(M)
// sine/cosine evaluations instead of 2 M; the product adds a few FP64 roundings).
void delay_ramp(const HostFrame& f, int p, std::vector<double2>& out) {
  constexpr int kB = 32;
  const int64_t MN = (int64_t)f.M * f.N;
  const int64_t nu = f.nu[p];
  auto phasor = [&](int64_t num) {
    num %= MN;
    if (num < 0) num += MN;
    const double ang = 2.0 * M_PI * ((double)num / (double)MN);
    return make_double2(std::cos(ang), std::sin(ang));
  };
  const int nl = f.M < kB ? f.M : kB;
  std::vector<double2> lo(nl);
  for (int kl = 0; kl < nl; ++kl) lo[kl] = phasor(nu * kl);
  const double hr = f.h[p].x, hi = f.h[p].y;
  for (int kh = 0; kh * kB < f.M; ++kh) {
    const double2 b = phasor(nu * ((int64_t)kh * kB - f.tau[p]));
    for (int kl = 0; kl < kB && kh * kB + kl < f.M; ++kl) {
      const double c = b.x * lo[kl].x - b.y * lo[kl].y;
      const double s = b.x * lo[kl].y + b.y * lo[kl].x;
      out.push_back(make_double2(hr * c - hi * s, hr * s + hi * c));
    }
  }
}

// Scalar fields of a frame descriptor: shape, regulariser, decision constants, solver
// options and staging geometry (from stage_geometry).
void frame_scalars(const HostFrame& fr, const otfs_cg_opts& o, int tiles, const FrameDev& geo,
                   FrameDev* d) {
  d->M = fr.M;
  d->N = fr.N;
  d->P = fr.P;
  d->T = tiles;
  d->lam = fr.lam;
  d->qside = fr.qam > 0 ? (int)std::lround(std::sqrt((double)fr.qam)) : 0;
  d->qscale = fr.qam > 0 ? (float)std::sqrt(2.0 * (fr.qam - 1) / 3.0) : 0.f;
  d->flags = (int32_t)o.flags;
  d->max_iters = o.max_iters;
  d->tol = o.rel_tol;
  d->refresh_every = o.refresh_every;
  d->skc = geo.skc;
  d->ssb = geo.ssb;
  d->swin = geo.swin;
  d->lpk = geo.lpk;
  d->lwc = geo.lwc;
  d->lwr = geo.lwr;
  d->tau_lo = geo.tau_lo;
  d->tau_hi = geo.tau_hi;
  d->nu_lo = geo.nu_lo;
  d->nu_hi = geo.nu_hi;
  d->resident = geo.resident;
  d->stream_t = (int64_t)fr.M * fr.N >= kStreamTElems ? 1 : 0;
  d->win_w = geo.win_w;
  d->win_rc = geo.win_rc;
  d->pcap = fr.P;
}

// Window of the LDS-windowed paired gathers for a frame cut into `tiles` row bands (of
// floor(N / tiles) or ceil(N / tiles) rows): frames whose rows split into 16-byte pairs (M a
// multiple of 128); the strip width is the gather rule's widest over the two band heights,
// the window width covers a strip, the delay range and an even origin, the height the
// tallest band and the Doppler range.  Returns the window's bytes, 0 (geometry untouched)
// if it does not fit the LDS budget.
int lds_pair_geometry(const HostFrame& f, int tiles, int budget_bytes, FrameDev* geo) {
  if (f.M % 128 != 0 || tiles < 1) return 0;
  const int dtau = geo->tau_hi - geo->tau_lo, dnu = geo->nu_hi - geo->nu_lo;
  const int band_lo = f.N / tiles, band_rows = (f.N + tiles - 1) / tiles;
  int kc = 0;
  for (int b : {band_lo, band_rows})
    kc = std::max(kc, 2 * strip_lanes_rule(f.M / 2, std::max(1, b)));
  int wc = kc + dtau + 1;
  wc += wc & 1;
  if (wc >= f.M) wc = f.M + 2;
  const int wr = band_rows + dnu >= f.N ? f.N : band_rows + dnu;
  const int64_t bytes = (int64_t)wr * wc * (int64_t)sizeof(float2);
  if (bytes > budget_bytes) return 0;
  geo->lpk = kc;
  geo->lwc = wc;
  geo->lwr = wr;
  return (int)bytes;
}

int lds_geometry(const HostFrame& f, int tiles, int band_rows, const otfs_cg_opts& o,
                 int budget_bytes, FrameDev* geo) {
  std::memset(geo, 0, sizeof(FrameDev));
  const int64_t E = (int64_t)f.M * f.N;
  const bool stored = stored_mode(o.flags) != kDNone;
  if ((o.flags & OTFS_LDS_GATHER) && !stored && tiles > 1) {
    stage_geometry(f, band_rows, 0, geo);   // shift ranges
    const int b = lds_pair_geometry(f, tiles, kLdsGatherBytes, geo);
    if (b > 0) return b;
  }
  if (tiles == 1 && !stored && o.refresh_every == 0 && !(o.flags & OTFS_NO_LDS_RESIDENT) &&
      E * kResidentVecs * (int64_t)sizeof(float2) <= kResidentBytes) {
    stage_geometry(f, band_rows, 0, geo);   // shift ranges only; no staging
    geo->resident = 1;
    return (int)(E * kResidentVecs * (int64_t)sizeof(float2));
  }
  if (stored) {
    stage_geometry(f, band_rows, 0, geo);
    return 0;
  }
  return stage_geometry(f, band_rows, budget_bytes / (int)sizeof(float2), geo) *
         (int)sizeof(float2);
}

int frame_kind(const FrameDev& geo) {
  if (geo.win_w > 0) return kKindWindowed;
  if (geo.lpk > 0) return kKindLds;
  return geo.resident ? kKindResident : (geo.skc > 0 ? kKindStaged : kKindDirect);
}

int refresh_lds_bytes(const std::vector<KindLaunch>& launches) {
  int b = 0;
  for (const KindLaunch& L : launches)
    if (L.kind == kKindLds) b = std::max(b, L.lds_bytes);
  return b;
}

int frame_lds_bytes(const HostFrame& f, const FrameDev& geo) {
  if (geo.win_w > 0)
    return win_lds_bytes(geo.win_w, geo.win_rc, geo.tau_hi - geo.tau_lo, geo.nu_hi - geo.nu_lo);
  if (geo.resident) return (int)((int64_t)f.M * f.N * kResidentVecs * (int64_t)sizeof(float2));
  if (geo.lpk > 0) return geo.lwr * geo.lwc * (int)sizeof(float2);
  if (geo.skc > 0) return kStageVecs * geo.swin * (int)sizeof(float2);
  return 0;
}

otfs_status plan_launches(const std::vector<HostFrame>& frames, const std::vector<FrameDev>& geo,
                          const std::vector<int>& tile_base, const std::vector<int>& tiles,
                          int sd, bool refresh, bool split_dir, int cus, int cap_override,
                          const XcdInfo& xi, bool agent, std::vector<int32_t>& qitems,
                          std::vector<int2>& qrange, std::vector<KindLaunch>& out) {
  qitems.clear();
  qrange.assign((size_t)kKinds * kMaxGroups, make_int2(0, 0));
  out.clear();
  // The H pass forms the direction inside its gathers when the direct frames have few
  // paths: the gathers then read two vectors, which costs more than the separate
  // direction pass saves once P is large (measured on the 16-path batches).
  bool fdir = sd == kDNone && !split_dir;
  for (size_t f = 0; f < frames.size(); ++f)
    if (frame_kind(geo[f]) == kKindDirect && frames[f].P > kFusedDirMaxPaths) fdir = false;
  auto kind_of = [&](size_t f) {
    const int k = frame_kind(geo[f]);
    return (k == kKindDirect && fdir) ? kKindDirectFD : k;
  };
  for (int kind = 0; kind < kKinds; ++kind) {
    std::vector<HostFrame> fs;
    std::vector<int> tb, tl;
    int lds = 0;
    for (size_t f = 0; f < frames.size(); ++f) {
      if (kind_of(f) != kind) continue;
      fs.push_back(frames[f]);
      tb.push_back(tile_base[f]);
      tl.push_back(tiles[f]);
      lds = std::max(lds, frame_lds_bytes(frames[f], geo[f]));
    }
    if (fs.empty()) continue;
    const int bpc = std::max(1, fused_blocks_per_cu(kind, sd, lds));
    int cap = bpc * cus;
    if (cap_override > 0) cap = std::min(cap, cap_override);
    KindLaunch L;
    L.kind = kind;
    L.nframes = (int)fs.size();
    L.lds_bytes = lds;
    L.qbase = kind * kMaxGroups;
    std::vector<int32_t> qi;
    std::vector<int2> qr;
    int per = 0;
    if (!agent && xi.round_robin && cap >= xi.nxcd &&
        make_queues(fs, tb, tl, xi.nxcd, cap / xi.nxcd, qi, qr, &per)) {
      L.xcd_local = true;
      L.ngroups = xi.nxcd;
      L.grid = per * xi.nxcd;
    } else if (make_queues(fs, tb, tl, 1, cap, qi, qr, &per)) {
      L.grid = per;
    } else {
      int maxT = 1;
      for (int t : tl) maxT = std::max(maxT, t);
      return fail(OTFS_E_UNSUPPORTED, "a frame needs %d cooperating workgroups but only %d fit",
                  maxT, cap);
    }
    const int base = (int)qitems.size();
    qitems.insert(qitems.end(), qi.begin(), qi.end());
    for (int g = 0; g < L.ngroups; ++g)
      qrange[(size_t)L.qbase + g] = make_int2(qr[g].x + base, qr[g].y + base);
    out.push_back(L);
  }
  return OTFS_OK;
}

// W[l] = e^{j 2 pi l / N}
void wrap_factors(const HostFrame& f, std::vector<double2>& out) {
  for (int l = 0; l < f.N; ++l) {
    const double ang = 2.0 * M_PI * ((double)l / (double)f.N);
    out.push_back(make_double2(std::cos(ang), std::sin(ang)));
  }
}

// ---------------------------------------------------------------------------------------
// tiling: frame f is split into T_f bands of Doppler rows, one workgroup each
// ---------------------------------------------------------------------------------------
#ifndef OTFS_FRAME_PAD
#define OTFS_FRAME_PAD 4160
#endif
// Elements left between consecutive frames in the workspace vectors (33 KiB, an odd
// number of 64-byte lines), so that the frames running together on one XCD do not start on
// the same memory-channel pattern; measured 2-3 % on the 64-frame batch.
constexpr int kFramePad = OTFS_FRAME_PAD;
static_assert(kFramePad % 2 == 0, "frame pad keeps pairs aligned");
// Element offset of frame f (at batch offset off) inside the workspace vectors: the batch
// offset plus f pads, rounded up to an even element.
static size_t frame_vec_offset(int64_t off, size_t f) {
  const size_t e = (size_t)off + f * (size_t)kFramePad;
  return e + (e & 1);
}
#ifndef OTFS_WG_PER_CU
#define OTFS_WG_PER_CU 2
#endif
int default_tile_elems(int64_t total_elems, int cus) {
  // aim at as many tiles as fused workgroups fit at once (OTFS_WG_PER_CU per CU)
  const int64_t target = std::max<int64_t>(1, (int64_t)cus * OTFS_WG_PER_CU);
  int64_t te = total_elems / target;
  te = std::max<int64_t>(te, 2048);
  te = std::min<int64_t>(te, 65536);
  return (int)te;
}

// Delay and Doppler shift ranges of a frame's paths, widened to contain 0.
static void shift_ranges(const HostFrame& f, int* tlo, int* thi, int* vlo, int* vhi) {
  *tlo = *thi = *vlo = *vhi = 0;
  for (int p = 0; p < f.P; ++p) {
    *tlo = std::min(*tlo, f.tau[p]);
    *thi = std::max(*thi, f.tau[p]);
    *vlo = std::min(*vlo, f.nu[p]);
    *vhi = std::max(*vhi, f.nu[p]);
  }
}

int window_width(const HostFrame& f, int w, int rc) {
  if (w <= 0 || rc <= 0) return 0;
  if (w % 64 != 0 || kBlock % w != 0 || f.M % w != 0) return 0;
  if (f.P > kWinPaths || rc > f.N) return 0;
  const int ty = kBlock / w;
  if (rc != 2 * ty && rc != 4 * ty) return 0;   // 2 or 4 output rows per thread and chunk
  int tlo, thi, vlo, vhi;
  shift_ranges(f, &tlo, &thi, &vlo, &vhi);
  const int dtau = thi - tlo, dnu = vhi - vlo;
  if (rc * ((w + dtau + 63) / 64) > kWaves * kWinLoads) return 0;
  if (win_lds_bytes(w, rc, dtau, dnu) > kMaxLdsBytes) return 0;
  return w;
}

void make_tiles(const std::vector<HostFrame>& frames, int tile_elems, std::vector<WorkItem>& items,
                std::vector<int>& tile_base, std::vector<int>& tiles, const std::vector<int>* winw) {
  items.clear();
  tile_base.assign(frames.size(), 0);
  tiles.assign(frames.size(), 0);
  for (size_t f = 0; f < frames.size(); ++f) {
    const HostFrame& fr = frames[f];
    const int w = winw ? (*winw)[f] : 0;
    if (w > 0) {   // windowed: strips of w delay columns over all rows
      tile_base[f] = (int)items.size();
      tiles[f] = fr.M / w;
      for (int t = 0; t < fr.M / w; ++t) {
        WorkItem it;
        it.frame = (int)f;
        it.tile = t;
        it.l_begin = 0;
        it.l_end = fr.N;
        it.k_begin = t * w;
        it.k_end = (t + 1) * w;
        items.push_back(it);
      }
      continue;
    }
    const int64_t E = (int64_t)fr.M * fr.N;
    int64_t T = (E + tile_elems / 2) / tile_elems;
    T = std::max<int64_t>(1, std::min<int64_t>(T, fr.N));
    tile_base[f] = (int)items.size();
    tiles[f] = (int)T;
    for (int t = 0; t < T; ++t) {
      WorkItem w;
      w.frame = (int)f;
      w.tile = t;
      w.l_begin = (int)((int64_t)t * fr.N / T);
      w.l_end = (int)((int64_t)(t + 1) * fr.N / T);
      w.k_begin = 0;
      w.k_end = fr.M;
      items.push_back(w);
    }
  }
}

bool make_queues(const std::vector<HostFrame>& frames, const std::vector<int>& tile_base,
                 const std::vector<int>& tiles, int ngroups, int per_group_cap,
                 std::vector<int32_t>& qitems, std::vector<int2>& qrange, int* per_group_grid) {
  qitems.clear();
  qrange.assign(kMaxGroups, make_int2(0, 0));
  *per_group_grid = 0;
  for (int t : tiles)
    if (t > per_group_cap) return false;
  // frames largest first, each to the least loaded group
  std::vector<int> order(frames.size());
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int f) {
    const HostFrame& fr = frames[f];
    return (double)fr.M * fr.N * (2.0 * fr.P + 6.0);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<std::vector<int32_t>> lists(ngroups);
  std::vector<double> load(ngroups, 0.0);
  for (int f : order) {
    int g = 0;
    for (int i = 1; i < ngroups; ++i)
      if (load[i] < load[g]) g = i;
    load[g] += work(f);
    for (int t = 0; t < tiles[f]; ++t) lists[g].push_back(tile_base[f] + t);
  }
  int per = 1;
  for (int g = 0; g < ngroups; ++g) {
    const int b = (int)qitems.size();
    qitems.insert(qitems.end(), lists[g].begin(), lists[g].end());
    qrange[g] = make_int2(b, (int)qitems.size());
    per = std::max(per, (int)lists[g].size());
  }
  *per_group_grid = std::min(per, per_group_cap);
  return true;
}

int stage_geometry(const HostFrame& f, int band_rows, int budget_elems, FrameDev* d) {
  // shift ranges, widened to contain 0 so that every output's own element is staged too
  int tlo = 0, thi = 0, vlo = 0, vhi = 0;
  for (int p = 0; p < f.P; ++p) {
    tlo = std::min(tlo, f.tau[p]);
    thi = std::max(thi, f.tau[p]);
    vlo = std::min(vlo, f.nu[p]);
    vhi = std::max(vhi, f.nu[p]);
  }
  d->tau_lo = tlo;
  d->tau_hi = thi;
  d->nu_lo = vlo;
  d->nu_hi = vhi;
  d->skc = 0;
  d->ssb = 0;
  d->swin = 0;
  if (budget_elems <= 0) return 0;
  const int dtau = thi - tlo, dnu = vhi - vlo;
  // column chunks of at most one workgroup width (one column per thread)
  int cands[6], nc = 0;
  if (f.M <= kBlock) cands[nc++] = f.M;
  for (int kc : {256, 128, 64, 32})
    if (kc < f.M) cands[nc++] = kc;
  double best = 1e300;
  int best_win = 0;
  for (int i = 0; i < nc; ++i) {
    const int kc = cands[i];
    const int tyc = kBlock / kc;
    const int sb = std::max(1, std::min(kStageRows * tyc, band_rows));
    const int wc = kc + dtau >= f.M ? f.M : kc + dtau;
    const int wr = sb + dnu >= f.N ? f.N : sb + dnu;
    const long long win = (long long)wr * ((wc + 31) / 32 * 32);   // rows padded to 32
    if (kStageVecs * win > budget_elems) continue;
    const double cost = (double)kStageVecs * win / ((double)sb * kc);
    if (cost < best - 1e-9) {
      best = cost;
      best_win = (int)win;
      d->skc = kc;
      d->ssb = sb;
      d->swin = (int)win;
    }
  }
  return d->skc > 0 ? kStageVecs * best_win : 0;
}

otfs_status probe_xcds(int device, void* scratch_dev, hipStream_t s, XcdInfo* out) {
  static std::mutex mu;
  static std::vector<int> cached_n(64, 0);
  static std::vector<int> cached_rr(64, 0);
  std::lock_guard<std::mutex> guard(mu);
  if (device >= 0 && device < 64 && cached_n[device] > 0) {
    out->nxcd = cached_n[device];
    out->round_robin = cached_rr[device] != 0;
    return OTFS_OK;
  }
  hipError_t e = launch_xcc_probe(static_cast<int*>(scratch_dev), kProbeBlocks, s);
  if (e != hipSuccess) return hip_fail(e, "XCC probe launch");
  std::vector<int> ids(kProbeBlocks, -1);
  if ((e = hipMemcpyAsync(ids.data(), scratch_dev, ids.size() * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "XCC probe readback");
  int mx = 0;
  bool ok = true;
  for (int v : ids) {
    if (v < 0 || v >= kMaxGroups) ok = false;
    mx = std::max(mx, v);
  }
  XcdInfo info;
  info.nxcd = ok ? mx + 1 : 1;
  info.round_robin = ok && info.nxcd > 1;
  for (int b = 0; b < kProbeBlocks && info.round_robin; ++b)
    if (ids[b] != b % info.nxcd) info.round_robin = false;
  if (device >= 0 && device < 64) {
    cached_n[device] = info.nxcd;
    cached_rr[device] = info.round_robin ? 1 : 0;
  }
  *out = info;
  return OTFS_OK;
}

// ---------------------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------------------
static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

void compute_layout(otfs_plan_t* pl) {
  Layout& L = pl->L;
  const size_t nf = pl->frames.size();
  size_t nitems = pl->items.size();
  size_t rt = 0, wt = 0, np = 0, dt = 0;
  for (auto& f : pl->frames) {
    rt += (size_t)f.P * f.M;
    wt += (size_t)f.N;
    np += (size_t)f.P;
    dt += (size_t)f.P * f.M * f.N;
  }
  const size_t E = (size_t)pl->total_elems;
  const bool refresh = pl->opts.refresh_every > 0;
  const int sd = stored_mode(pl->opts.flags);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.frames = take(nf * sizeof(FrameDev));
  L.items = take(nitems * sizeof(WorkItem));
  L.qitems = take(nitems * sizeof(int32_t));
  L.qrange = take(kKinds * kMaxGroups * sizeof(int2));
  L.qhead = take(kKinds * kMaxGroups * sizeof(unsigned));
  L.probe = take(kProbeBlocks * sizeof(int));
  L.rtab = take(rt * sizeof(float2));
  L.wtab = take(wt * sizeof(float2));
  L.rtab64 = refresh ? take(rt * sizeof(double2)) : 0;
  L.wtab64 = refresh ? take(wt * sizeof(double2)) : 0;
  L.paths = take(np * sizeof(int2));
  L.part_pa = take(nitems * sizeof(float));
  L.part_cc = take(nitems * sizeof(float));
  L.part_d = take(nitems * sizeof(double));
  L.bar = take(nf * sizeof(unsigned));
  L.prog = take(nitems * sizeof(unsigned));
  L.st = take(nf * sizeof(FrameState));
  L.abort = take(sizeof(unsigned));
  // frames staggered, each starting at an even element (16-byte aligned pairs)
  const size_t Ep = E + pl->frames.size() * (size_t)(kFramePad + 1);
  L.c = take(Ep * sizeof(float2));
  L.p0 = take(Ep * sizeof(float2));
  L.p1 = take(Ep * sizeof(float2));
  L.t = take(Ep * sizeof(float2));
  L.a = take(Ep * sizeof(float2));
  L.u = refresh ? take(Ep * sizeof(float2)) : 0;
  L.dtab = sd == kDNone ? 0 : take(dt * (sd == kDC64 ? sizeof(float2) : sizeof(uint32_t)));
  L.total = std::max<size_t>(o, 256);
}

// Per-frame window widths, tiles and workspace layout after a change of the tiling or the
// windowed form.
void retile(otfs_plan_t* pl) {
  pl->winw.assign(pl->frames.size(), 0);
  // the windowed kind synthesises D and has no refresh passes: those modes keep row bands
  const bool win_ok = stored_mode(pl->opts.flags) == kDNone && pl->opts.refresh_every == 0;
  for (size_t f = 0; f < pl->frames.size() && win_ok; ++f)
    pl->winw[f] = window_width(pl->frames[f], pl->win_w_req, pl->win_rc_req);
  make_tiles(pl->frames, pl->tile_elems, pl->items, pl->tile_base, pl->tiles, &pl->winw);
  compute_layout(pl);
}

}  // namespace otfs

using namespace otfs;

// =========================================================================================
// C ABI
// =========================================================================================
extern "C" const char* otfs_last_error(void) { return otfs::last_error(); }

#ifndef OTFS_SOURCE_SHA
#define OTFS_SOURCE_SHA "unstamped"
#endif
#ifndef OTFS_BUILD_ARCH
#define OTFS_BUILD_ARCH "unknown"
#endif
extern "C" const char* otfs_build_info(void) {
  return "source_sha=" OTFS_SOURCE_SHA " arch=" OTFS_BUILD_ARCH;
}

extern "C" otfs_status otfs_plan(const otfs_frame_desc* frames, int32_t nframes,
                                 const otfs_cg_opts* opts, otfs_plan_t** out) {
  if (!out) return fail(OTFS_E_INVAL, "out must be non-null");
  *out = nullptr;
  if (nframes < 0) return fail(OTFS_E_INVAL, "nframes must be >= 0");
  if (nframes > 0 && !frames) return fail(OTFS_E_INVAL, "frames is null");
  otfs_plan_t* pl = new (std::nothrow) otfs_plan_t();
  if (!pl) return fail(OTFS_E_NOMEM, "out of host memory");
  otfs_status st = validate_opts(opts, &pl->opts);
  if (st != OTFS_OK) {
    delete pl;
    return st;
  }
  pl->frames.resize(nframes);
  int64_t total = 0;
  int maxp = 0;
  for (int i = 0; i < nframes; ++i) {
    st = validate_frame(frames[i], i, &pl->frames[i]);
    if (st != OTFS_OK) {
      delete pl;
      return st;
    }
    pl->frames[i].off = total;
    total += (int64_t)frames[i].M * frames[i].N;
    maxp = std::max(maxp, frames[i].P);
  }
  pl->total_elems = total;
  pl->max_paths = maxp;
  int cus = 256;
  int dev = 0, ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 && hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  (void)hipGetLastError();
  pl->cus = cus;
  pl->tile_elems = default_tile_elems(total, cus);
  retile(pl);
  *out = pl;
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_workspace_bytes(const otfs_plan_t* plan, size_t* bytes,
                                                 int64_t* total_elems) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (bytes) *bytes = plan->L.total;
  if (total_elems) *total_elems = plan->total_elems;
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_info(const otfs_plan_t* plan, otfs_plan_info_t* info) {
  if (!plan || !info) return fail(OTFS_E_INVAL, "plan and info must be non-null");
  info->nframes = (int32_t)plan->frames.size();
  info->total_elems = plan->total_elems;
  info->grid = 0;
  info->block = kBlock;
  info->max_paths = plan->max_paths;
  info->tile_elems = plan->tile_elems;
  info->groups = 0;
  info->xcd_local = plan->launches.empty() ? 0 : 1;
  info->lds_bytes = 0;
  for (const KindLaunch& L : plan->launches) {
    info->grid += L.grid;
    info->groups = std::max(info->groups, L.ngroups);
    info->xcd_local = info->xcd_local && L.xcd_local ? 1 : 0;
    info->lds_bytes = std::max(info->lds_bytes, L.lds_bytes);
  }
  info->launches = (int32_t)plan->launches.size();
  info->fused_direction_frames = 0;
  for (const KindLaunch& L : plan->launches)
    if (L.kind == kKindDirectFD) info->fused_direction_frames += L.nframes;
  info->staged_frames = 0;
  info->resident_frames = 0;
  for (const FrameDev& d : plan->h_frames) {
    info->staged_frames += (d.skc > 0 || d.lpk > 0) ? 1 : 0;
    info->resident_frames += d.resident ? 1 : 0;
  }
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_set_tiling(otfs_plan_t* plan, int32_t tile_elems,
                                            int32_t max_grid) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (tile_elems < 0 || max_grid < 0)
    return fail(OTFS_E_INVAL, "tile_elems and max_grid must be >= 0");
  plan->tile_elems = tile_elems > 0 ? tile_elems : default_tile_elems(plan->total_elems, plan->cus);
  plan->max_grid_req = max_grid;
  retile(plan);
  plan->bound = false;
  plan->drop_graph();
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_set_window(otfs_plan_t* plan, int32_t strip_cols,
                                            int32_t chunk_rows) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (strip_cols < 0 || chunk_rows < 0)
    return fail(OTFS_E_INVAL, "strip_cols and chunk_rows must be >= 0");
  plan->win_w_req = strip_cols > 0 && chunk_rows > 0 ? strip_cols : 0;
  plan->win_rc_req = strip_cols > 0 && chunk_rows > 0 ? chunk_rows : 0;
  retile(plan);
  plan->bound = false;
  plan->drop_graph();
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_set_staging(otfs_plan_t* plan, int32_t lds_bytes) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (lds_bytes < 0 || lds_bytes > 65536)
    return fail(OTFS_E_INVAL, "lds_bytes must be in [0, 65536] (got %d)", lds_bytes);
  plan->stage_bytes = lds_bytes;
  plan->bound = false;
  plan->drop_graph();
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_bind(otfs_plan_t* plan, void* ws, size_t ws_bytes, void* stream) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (!ws && plan->L.total > 0) return fail(OTFS_E_INVAL, "workspace is null");
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return fail(OTFS_E_INVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < plan->L.total)
    return fail(OTFS_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, plan->L.total);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  plan->device = dev;
  plan->drop_graph();

  // LDS use per frame: resident vectors or staged-gather windows (decides the launch kind
  // of every frame and the dynamic LDS of each launch)
  std::vector<FrameDev> geo(plan->frames.size());
  for (size_t f = 0; f < plan->frames.size(); ++f) {
    int band = 1;
    for (int t = 0; t < plan->tiles[f]; ++t) {
      const WorkItem& w = plan->items[plan->tile_base[f] + t];
      band = std::max(band, w.l_end - w.l_begin);
    }
    lds_geometry(plan->frames[f], plan->tiles[f], band, plan->opts, plan->stage_bytes, &geo[f]);
    if (plan->winw[f] > 0) {   // windowed strips: no staging, not resident
      geo[f].resident = 0;
      geo[f].skc = geo[f].ssb = geo[f].swin = 0;
      geo[f].win_w = plan->winw[f];
      geo[f].win_rc = plan->win_rc_req;
    }
  }

  // work queues of the fused kernel (need the occupancy and XCD layout of this device)
  int cus = plan->cus;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    cus = v;
  XcdInfo xi;
  otfs_status pst = probe_xcds(dev, static_cast<char*>(ws) + plan->L.probe, s, &xi);
  if (pst != OTFS_OK) return pst;
  plan->ref_xcds = xi.round_robin ? xi.nxcd : 1;
  pst = plan_launches(plan->frames, geo, plan->tile_base, plan->tiles,
                      stored_mode(plan->opts.flags), plan->opts.refresh_every > 0,
                      (plan->opts.flags & OTFS_SPLIT_DIRECTION) != 0, cus, plan->max_grid_req, xi,
                      (plan->opts.flags & OTFS_AGENT_BARRIER) != 0,
                      plan->qitems, plan->qrange, plan->launches);
  if (pst != OTFS_OK) return pst;

  // host tables
  const Layout& L = plan->L;
  char* base = static_cast<char*>(ws);
  std::vector<double2> r64, w64;
  std::vector<int2> paths;
  std::vector<FrameDev> fd(plan->frames.size());
  size_t ro = 0, wo = 0, po = 0, dto = 0;
  const bool refresh = plan->opts.refresh_every > 0;
  const int sd = stored_mode(plan->opts.flags);
  const size_t dsz = sd == kDC64 ? sizeof(float2) : sizeof(uint32_t);
  for (size_t f = 0; f < plan->frames.size(); ++f) {
    const HostFrame& fr = plan->frames[f];
    FrameDev& d = fd[f];
    std::memset(&d, 0, sizeof d);
    for (int p = 0; p < fr.P; ++p) delay_ramp(fr, p, r64);
    wrap_factors(fr, w64);
    for (int p = 0; p < fr.P; ++p) paths.push_back(make_int2(fr.tau[p], fr.nu[p]));
    const size_t E = (size_t)fr.M * fr.N;
    const size_t eo = frame_vec_offset(fr.off, f);
    d.c = reinterpret_cast<float2*>(base + L.c) + eo;
    d.p0 = reinterpret_cast<float2*>(base + L.p0) + eo;
    d.p1 = reinterpret_cast<float2*>(base + L.p1) + eo;
    d.t = reinterpret_cast<float2*>(base + L.t) + eo;
    d.a = reinterpret_cast<float2*>(base + L.a) + eo;
    d.u = refresh ? reinterpret_cast<float2*>(base + L.u) + eo : nullptr;
    d.rtab = reinterpret_cast<const float2*>(base + L.rtab) + ro;
    d.wtab = reinterpret_cast<const float2*>(base + L.wtab) + wo;
    d.rtab64 = refresh ? reinterpret_cast<const double2*>(base + L.rtab64) + ro : nullptr;
    d.wtab64 = refresh ? reinterpret_cast<const double2*>(base + L.wtab64) + wo : nullptr;
    d.paths = reinterpret_cast<const int2*>(base + L.paths) + po;
    d.dtab = sd != kDNone ? static_cast<const void*>(base + L.dtab + dto * dsz) : nullptr;
    const int tb = plan->tile_base[f];
    d.part_pa = reinterpret_cast<float*>(base + L.part_pa) + tb;
    d.part_cc = reinterpret_cast<float*>(base + L.part_cc) + tb;
    d.part_d = reinterpret_cast<double*>(base + L.part_d) + tb;
    d.bar = reinterpret_cast<unsigned*>(base + L.bar) + f;
    d.prog = reinterpret_cast<unsigned*>(base + L.prog) + tb;
    d.st = reinterpret_cast<FrameState*>(base + L.st) + f;
    frame_scalars(fr, plan->opts, plan->tiles[f], geo[f], &d);
    d.off = fr.off;
    d.index = (int32_t)f;
    ro += (size_t)fr.P * fr.M;
    wo += (size_t)fr.N;
    po += (size_t)fr.P;
    dto += (size_t)fr.P * E;
  }
  plan->h_rtab.resize(r64.size());
  plan->h_wtab.resize(w64.size());
  for (size_t i = 0; i < r64.size(); ++i) plan->h_rtab[i] = make_float2((float)r64[i].x, (float)r64[i].y);
  for (size_t i = 0; i < w64.size(); ++i) plan->h_wtab[i] = make_float2((float)w64[i].x, (float)w64[i].y);
  plan->h_rtab64 = refresh ? r64 : std::vector<double2>();
  plan->h_wtab64 = refresh ? w64 : std::vector<double2>();
  plan->h_paths = paths;
  plan->h_frames = fd;

  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  if ((e = up(L.frames, fd.data(), fd.size() * sizeof(FrameDev))) != hipSuccess ||
      (e = up(L.items, plan->items.data(), plan->items.size() * sizeof(WorkItem))) != hipSuccess ||
      (e = up(L.qitems, plan->qitems.data(), plan->qitems.size() * sizeof(int32_t))) != hipSuccess ||
      (e = up(L.qrange, plan->qrange.data(), plan->qrange.size() * sizeof(int2))) != hipSuccess ||
      (e = up(L.rtab, plan->h_rtab.data(), plan->h_rtab.size() * sizeof(float2))) != hipSuccess ||
      (e = up(L.wtab, plan->h_wtab.data(), plan->h_wtab.size() * sizeof(float2))) != hipSuccess ||
      (e = up(L.paths, plan->h_paths.data(), plan->h_paths.size() * sizeof(int2))) != hipSuccess)
    return hip_fail(e, "hipMemcpyAsync (plan tables)");
  if (refresh) {
    if ((e = up(L.rtab64, plan->h_rtab64.data(), plan->h_rtab64.size() * sizeof(double2))) != hipSuccess ||
        (e = up(L.wtab64, plan->h_wtab64.data(), plan->h_wtab64.size() * sizeof(double2))) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync (FP64 tables)");
  }
  plan->ws = ws;
  plan->d_frames = reinterpret_cast<FrameDev*>(base + L.frames);
  plan->d_items = reinterpret_cast<WorkItem*>(base + L.items);
  plan->d_qitems = reinterpret_cast<int32_t*>(base + L.qitems);
  plan->d_qrange = reinterpret_cast<int2*>(base + L.qrange);
  plan->d_qhead = reinterpret_cast<unsigned*>(base + L.qhead);
  plan->d_abort = reinterpret_cast<unsigned*>(base + L.abort);
  if (sd != kDNone) {
    if ((e = launch_build_d(sd, plan->d_frames, plan->d_items, (int)plan->items.size(), s)) != hipSuccess)
      return hip_fail(e, "build D");
  }
  // the host arrays above must outlive the copies
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize (bind)");
  plan->bound = true;
  plan->device_paths = false;   // the tables just uploaded are the host's
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_free(otfs_plan_t* plan) {
  if (!plan) return OTFS_OK;
  plan->drop_graph();
  if (plan->ev_begin) (void)hipEventDestroy(plan->ev_begin);
  if (plan->ev_end) (void)hipEventDestroy(plan->ev_end);
  delete plan;
  return OTFS_OK;
}

static otfs_status check_bound(const otfs_plan_t* plan) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (!plan->bound) return fail(OTFS_E_STATE, "plan is not bound to a workspace (otfs_plan_bind)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
    return fail(OTFS_E_STATE, "current device %d differs from the bound device %d", dev, plan->device);
  return OTFS_OK;
}

static otfs_status apply_common(const otfs_plan_t* plan, bool adj, const void* in, void* out,
                                void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (plan->total_elems == 0) return OTFS_OK;
  if (!in || !out) return fail(OTFS_E_INVAL, "input and output must be non-null");
  if (in == out) return fail(OTFS_E_INVAL, "input and output must be distinct buffers");
  const int sd = stored_mode(plan->opts.flags);
  int lds = 0;   // staged frames stage their windows here too, windowed frames their rings
  for (const KindLaunch& L : plan->launches)
    if (L.kind == kKindStaged) lds = L.lds_bytes;
  for (const FrameDev& d : plan->h_frames)
    if (d.win_w > 0)
      lds = std::max(lds, win_lds_bytes(d.win_w, d.win_rc, d.tau_hi - d.tau_lo, d.nu_hi - d.nu_lo));
  hipError_t e = launch_apply(adj, sd, plan->d_frames, plan->d_items, (int)plan->items.size(),
                              static_cast<const float2*>(in), static_cast<float2*>(out), lds,
                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, adj ? "apply H^H" : "apply H");
  return OTFS_OK;
}

extern "C" otfs_status otfs_apply_H(const otfs_plan_t* plan, const void* x, void* y, void* stream) {
  return apply_common(plan, false, x, y, stream);
}
extern "C" otfs_status otfs_apply_HH(const otfs_plan_t* plan, const void* y, void* x, void* stream) {
  return apply_common(plan, true, y, x, stream);
}

// Number of fused launches of one solve: with the FP64 refresh every k iterations, frames
// leave the fused launch after iterations k, 2k, ... below the cap for the refresh
// launches, so the solve is floor((max_iters - 1) / k) + 1 fused segments.
static int fused_segments(const otfs_cg_opts& o) {
  return o.refresh_every > 0 ? (o.max_iters - 1) / o.refresh_every + 1 : 1;
}

// the launch sequence of one fused solve: reset, then per segment the persistent kernel of
// every launch kind followed by the refresh launches (optionally timed as a whole)
static hipError_t enqueue_fused(otfs_plan_t* plan, const Bases& B, hipStream_t s, bool timed) {
  hipError_t e = launch_reset(plan->d_frames, (int)plan->frames.size(), plan->d_abort,
                              plan->d_qhead, kKinds * kMaxGroups, s);
  if (e != hipSuccess) return e;
  if (timed && (e = hipEventRecord(plan->ev_begin, s)) != hipSuccess) return e;
  // Frames of the windowed-pairs kind refresh inside the fused launch when their windows
  // fit; with the host's path tables (for which the plan sized the windows) and every frame
  // of that kind, one launch runs the whole solve.
  bool inline_refresh = !plan->device_paths && !plan->launches.empty();
  for (const KindLaunch& L : plan->launches) inline_refresh = inline_refresh && L.kind == kKindLds;
  const int nseg = inline_refresh ? 1 : fused_segments(plan->opts);
  for (int seg = 0; seg < nseg; ++seg) {
    for (const KindLaunch& L : plan->launches) {
      e = launch_cg_fused(L.kind, stored_mode(plan->opts.flags), plan->d_frames, plan->d_items,
                          plan->d_qitems, plan->d_qrange + L.qbase, plan->d_qhead + L.qbase,
                          L.ngroups, L.grid, plan->opts.max_iters, B, L.xcd_local,
                          plan->d_abort, L.lds_bytes, plan->wait_us, s);
      if (e != hipSuccess) return e;
    }
    if (seg + 1 < nseg) {
      e = launch_refresh(plan->d_frames, plan->d_items, (int)plan->items.size(), B,
                         plan->d_qhead, kKinds * kMaxGroups, refresh_lds_bytes(plan->launches),
                         plan->ref_xcds, s);
      if (e != hipSuccess) return e;
    }
  }
  if (timed && (e = hipEventRecord(plan->ev_end, s)) != hipSuccess) return e;
  return hipSuccess;
}

extern "C" otfs_status otfs_lmmse_cg(otfs_plan_t* plan, const void* y, void* xhat, uint8_t* sym,
                                     otfs_frame_stats* stats, void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (plan->frames.empty()) return OTFS_OK;
  if (!y || !xhat) return fail(OTFS_E_INVAL, "y and xhat must be non-null");
  if (y == xhat) return fail(OTFS_E_INVAL, "y and xhat must be distinct buffers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Bases B{y, static_cast<float2*>(xhat), sym, stats};
  const bool timed = (plan->opts.flags & OTFS_TIME_KERNEL) != 0;
  hipError_t e;
  if (timed && !plan->ev_begin) {
    if ((e = hipEventCreate(&plan->ev_begin)) != hipSuccess || (e = hipEventCreate(&plan->ev_end)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
  }
  if ((plan->opts.flags & OTFS_USE_GRAPH) && !timed) {
    if (s == nullptr)
      return fail(OTFS_E_INVAL, "OTFS_USE_GRAPH needs a created stream (the NULL stream cannot be captured)");
    const GraphKey key{y, xhat, sym, stats, s};
    if (!plan->gexec || !(plan->gkey == key)) {
      plan->drop_graph();
      if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
      hipError_t le = enqueue_fused(plan, B, s, false);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(s, &g);
      if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "capture of the fused CG launch");
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        plan->gexec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
      }
      plan->gkey = key;
    }
    if ((e = hipGraphLaunch(plan->gexec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return OTFS_OK;
  }
  if ((e = enqueue_fused(plan, B, s, timed)) != hipSuccess) return hip_fail(e, "fused CG launch");
  plan->timed_pending = timed;
  return OTFS_OK;
}

extern "C" otfs_status otfs_lmmse_cg_plain(otfs_plan_t* plan, const void* y, void* xhat,
                                           uint8_t* sym, otfs_frame_stats* stats, void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (plan->frames.empty()) return OTFS_OK;
  if (!y || !xhat) return fail(OTFS_E_INVAL, "y and xhat must be non-null");
  if (y == xhat) return fail(OTFS_E_INVAL, "y and xhat must be distinct buffers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Bases B{y, static_cast<float2*>(xhat), sym, stats};
  if (stored_mode(plan->opts.flags) != kDNone)
    return fail(OTFS_E_UNSUPPORTED, "the plain form synthesises D on the fly only");
  hipError_t e = launch_reset(plan->d_frames, (int)plan->frames.size(), plan->d_abort,
                              plan->d_qhead, kKinds * kMaxGroups, s);
  if (e != hipSuccess) return hip_fail(e, "reset");
  for (size_t f = 0; f < plan->frames.size(); ++f) {
    e = launch_plain_frame(plan->d_frames, (int)f, plan->d_items, plan->tile_base[f],
                           plan->tiles[f], plan->opts.max_iters, B, s);
    if (e != hipSuccess) return hip_fail(e, "plain CG launch");
  }
  return OTFS_OK;
}

extern "C" otfs_status otfs_dzt(int32_t M, int32_t N, int32_t nframes, const void* in, void* out,
                                int32_t inverse, void* stream) {
  if (M < 1 || N < 1 || nframes < 0)
    return fail(OTFS_E_INVAL, "need M, N >= 1 and nframes >= 0 (got %d, %d, %d)", M, N, nframes);
  if ((int64_t)M * N > (int64_t(1) << 28))
    return fail(OTFS_E_INVAL, "M*N = %lld exceeds 2^28", (long long)M * N);
  if (N > kDztMaxN)
    return fail(OTFS_E_UNSUPPORTED, "N = %d exceeds %d (twiddle table in LDS)", N, kDztMaxN);
  if (nframes == 0) return OTFS_OK;
  if (!in || !out) return fail(OTFS_E_INVAL, "in and out must be non-null");
  if (in == out) return fail(OTFS_E_INVAL, "in and out must be distinct buffers");
  hipError_t e = launch_dzt(M, N, nframes, inverse != 0, static_cast<const float2*>(in),
                            static_cast<float2*>(out), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "DZT");
  return OTFS_OK;
}

extern "C" otfs_status otfs_bit_errors(const otfs_plan_t* plan, const uint8_t* sym,
                                       const uint8_t* sym_tx, uint64_t* errs, void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (plan->frames.empty()) return OTFS_OK;
  if (!sym || !sym_tx || !errs) return fail(OTFS_E_INVAL, "sym, sym_tx and errs must be non-null");
  hipError_t e = launch_bit_errors(plan->d_frames, plan->d_items, (int)plan->items.size(), sym,
                                   sym_tx, reinterpret_cast<unsigned long long*>(errs),
                                   (int)plan->frames.size(), true, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "bit errors");
  return OTFS_OK;
}

extern "C" otfs_status otfs_lmmse_cg_trace(otfs_plan_t* plan, const void* y, void* xhat,
                                           uint8_t* sym, otfs_frame_stats* stats,
                                           const uint8_t* sym_tx, uint64_t* errs, void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (plan->frames.empty()) return OTFS_OK;
  if (!y || !xhat || !sym || !sym_tx || !errs)
    return fail(OTFS_E_INVAL, "y, xhat, sym, sym_tx and errs must be non-null");
  if (y == xhat) return fail(OTFS_E_INVAL, "y and xhat must be distinct buffers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Bases B{y, static_cast<float2*>(xhat), sym, stats};
  const int nf = (int)plan->frames.size(), ni = (int)plan->items.size();
  auto* ue = reinterpret_cast<unsigned long long*>(errs);
  hipError_t e = launch_reset(plan->d_frames, nf, plan->d_abort, plan->d_qhead, kKinds * kMaxGroups, s);
  if (e == hipSuccess) e = launch_fill_u64(ue, (int64_t)plan->opts.max_iters * nf, s);
  for (int it = 0; it < plan->opts.max_iters && e == hipSuccess; ++it) {
    if (it > 0) {   // counters and cursors of the next one-iteration launch
      e = plan->opts.refresh_every > 0
              ? launch_refresh(plan->d_frames, plan->d_items, ni, B, plan->d_qhead,
                               kKinds * kMaxGroups, refresh_lds_bytes(plan->launches),
                               plan->ref_xcds, s)
              : launch_step_reset(plan->d_frames, nf, plan->d_abort, plan->d_qhead,
                                  kKinds * kMaxGroups, s);
    }
    for (const KindLaunch& L : plan->launches) {
      if (e != hipSuccess) break;
      e = launch_cg_fused(L.kind, stored_mode(plan->opts.flags), plan->d_frames, plan->d_items,
                          plan->d_qitems, plan->d_qrange + L.qbase, plan->d_qhead + L.qbase,
                          L.ngroups, L.grid, 1, B, L.xcd_local, plan->d_abort, L.lds_bytes,
                          plan->wait_us, s);
    }
    if (e == hipSuccess)
      e = launch_trace_errors(plan->d_frames, plan->d_items, ni, B, sym_tx, ue + (size_t)it * nf, s);
  }
  if (e != hipSuccess) return hip_fail(e, "CG trace");
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_get_paths(const otfs_plan_t* plan, int32_t frame,
                                           int32_t capacity, int32_t* P, int32_t* delay,
                                           int32_t* doppler, float* h, void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (frame < 0 || frame >= (int32_t)plan->frames.size())
    return fail(OTFS_E_INVAL, "frame %d out of range [0, %zu)", frame, plan->frames.size());
  if (!P || (capacity > 0 && (!delay || !doppler || !h)) || capacity < 0)
    return fail(OTFS_E_INVAL, "P must be non-null; delay, doppler, h non-null when capacity > 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  FrameDev d;
  hipError_t e = hipMemcpyAsync(&d, plan->d_frames + frame, sizeof d, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "path table readback");
  *P = d.P;
  const int n = std::min(d.P, capacity);
  if (n > 0) {
    std::vector<int2> tn(n);
    std::vector<float2> r(n);   // R_p[tau_p mod M] = h_p (the ramp's phase vanishes at k = tau_p)
    e = hipMemcpyAsync(tn.data(), d.paths, n * sizeof(int2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int p = 0; p < n && e == hipSuccess; ++p) {
      const int k = ((tn[p].x % d.M) + d.M) % d.M;
      e = hipMemcpyAsync(&r[p], d.rtab + (size_t)p * d.M + k, sizeof(float2), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "path table readback");
    const int64_t MN = (int64_t)d.M * d.N;
    for (int p = 0; p < n; ++p) {
      delay[p] = tn[p].x;
      doppler[p] = tn[p].y;
      // R_p[k] = h_p e^{j 2 pi nu (k - tau) / MN}; k - tau is 0 (tau >= 0) or M (tau < 0)
      const int k = ((tn[p].x % d.M) + d.M) % d.M;
      int64_t num = ((int64_t)tn[p].y * (k - tn[p].x)) % MN;
      if (num < 0) num += MN;
      const double ang = -2.0 * M_PI * ((double)num / (double)MN);
      const double c = std::cos(ang), sn = std::sin(ang);
      h[2 * p] = (float)(r[p].x * c - r[p].y * sn);
      h[2 * p + 1] = (float)(r[p].x * sn + r[p].y * c);
    }
  }
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_paths_from_pilot(otfs_plan_t* plan, const void* ypilot,
                                                  float theta, int32_t* npaths, void* stream) {
  otfs_status st = check_bound(plan);
  if (st != OTFS_OK) return st;
  if (plan->frames.empty()) return OTFS_OK;
  if (!ypilot) return fail(OTFS_E_INVAL, "ypilot must be non-null");
  if (!(theta >= 0.f) || !std::isfinite(theta))
    return fail(OTFS_E_INVAL, "theta must be finite and >= 0");
  for (const FrameDev& d : plan->h_frames)
    if (d.skc > 0 || d.win_w > 0)
      return fail(OTFS_E_UNSUPPORTED,
                  "frames with LDS-staged or windowed gathers keep the windows planned on the "
                  "host from their given paths");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_pilot_paths(plan->d_frames, (int)plan->frames.size(),
                                    static_cast<const float2*>(ypilot), theta, npaths, s);
  if (e != hipSuccess) return hip_fail(e, "pilot path estimation");
  plan->device_paths = true;
  const int sd = stored_mode(plan->opts.flags);
  if (sd != kDNone &&
      (e = launch_build_d(sd, plan->d_frames, plan->d_items, (int)plan->items.size(), s)) != hipSuccess)
    return hip_fail(e, "build D");
  return OTFS_OK;
}

extern "C" otfs_status otfs_lmmse_cg_noalloc(otfs_plan_t* plan, const void* y, void* xhat,
                                             uint8_t* sym, otfs_frame_stats* stats, void* stream) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  if (plan->opts.flags & (OTFS_USE_GRAPH | OTFS_TIME_KERNEL))
    return fail(OTFS_E_UNSUPPORTED,
                "otfs_lmmse_cg_noalloc runs without OTFS_USE_GRAPH and OTFS_TIME_KERNEL");
  if (plan->L.total > kNoAllocBytes)
    return fail(OTFS_E_NOMEM,
                "the plan needs a workspace of %zu bytes; the static scratch holds %zu bytes",
                plan->L.total, kNoAllocBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  void* ws = nullptr;
  if ((e = noalloc_scratch(dev, &ws)) != hipSuccess)
    return hip_fail(e, "hipGetSymbolAddress (scratch)");
  // every call rebinds: the scratch is shared by all calls on this device and holds the
  // tables of whichever plan used it last
  otfs_status st = otfs_plan_bind(plan, ws, kNoAllocBytes, stream);
  if (st != OTFS_OK) return st;
  return otfs_lmmse_cg(plan, y, xhat, sym, stats, stream);
}

extern "C" otfs_status otfs_plan_set_wait_limit(otfs_plan_t* plan, int64_t wait_us) {
  if (!plan) return fail(OTFS_E_INVAL, "plan is null");
  plan->wait_us = wait_us < 0 ? -1 : wait_us;
  plan->drop_graph();
  return OTFS_OK;
}

extern "C" otfs_status otfs_plan_kernel_ms(otfs_plan_t* plan, float* ms) {
  if (!plan || !ms) return fail(OTFS_E_INVAL, "plan and ms must be non-null");
  if (!plan->timed_pending || !plan->ev_begin)
    return fail(OTFS_E_STATE, "no timed otfs_lmmse_cg call (set OTFS_TIME_KERNEL)");
  hipError_t e = hipEventSynchronize(plan->ev_end);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  if ((e = hipEventElapsedTime(ms, plan->ev_begin, plan->ev_end)) != hipSuccess)
    return hip_fail(e, "hipEventElapsedTime");
  return OTFS_OK;
}
