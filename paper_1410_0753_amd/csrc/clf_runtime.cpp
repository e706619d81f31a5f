// Host runtime and C-ABI of the split-step library (see include/clf.h).
//
// Responsibilities: argument validation, the one-time depth preprocessing
// (section Numerical stability: dstab, newdw, newdc), metric arrays
// (inverse spacings, spherical row factors and tan(lat)/R), the still-water
// Courant check (stability remark after solver2), carving of the caller's
// workspace, the tile list of the march kernel, and the per-step launch
// sequence (forcing ring -> fused step -> sampling) on the caller's stream.

#include "clf.h"
#include "clf_internal.h"

#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace clf;

namespace {

// Host trace ranges (roctx) around the library's calls, seen by a profiler
// (rocprofv3 --marker-trace).  The roctx library is looked up once at run
// time; without it the ranges cost nothing and the library has no link-time
// dependency on it.
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};

const Roctx& roctx() {
  static Roctx r = [] {
    Roctx t;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    if (h) {
      t.push = (int (*)(const char*))dlsym(h, "roctxRangePushA");
      t.pop = (int (*)())dlsym(h, "roctxRangePop");
      if (!t.push || !t.pop) t.push = nullptr, t.pop = nullptr;
    }
    return t;
  }();
  return r;
}

struct TraceRange {
  explicit TraceRange(const char* name) {
    if (roctx().push) roctx().push(name);
  }
  ~TraceRange() {
    if (roctx().pop) roctx().pop();
  }
};

}  // namespace

namespace {

const bool kHaveFp32Kernels = true;
const double kGrav = 9.81;
const double kPiD = 3.14159265358979323846;

thread_local std::string g_init_error;

struct Enc {
  int nx, ny;
  int off[4];  // offset of each side block inside a record
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  size_t gd, st, sd, fd, tiles, f[9], xib, xisb, xfac, yib, yisb, tanR, gidx, gtab, grec, sidx, swt,
      sout, srec, ft[4], fv[4], total;
  int ntiles_max;
};

int strips_of(int nx) { return (nx + STRIP - 1) / STRIP; }

constexpr int kMinSeg = 8;

Layout plan(int nx, int ny, const clf_params& p) {
  Layout L{};
  const size_t es = p.precision == CLF_FP32 ? 4 : 8;
  const size_t N = (size_t)nx * ny;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.gd = take(sizeof(GridDesc));
  L.st = take(sizeof(StepState));
  L.sd = take(sizeof(SampleDesc));
  L.fd = take(sizeof(ForceDesc));
  L.ntiles_max = strips_of(nx) * ((ny + kMinSeg - 1) / kMinSeg) + 8 * WAVES_PER_BLOCK * 2;
  L.tiles = take(sizeof(Tile) * (size_t)L.ntiles_max);
  for (int i = 0; i < 9; ++i) L.f[i] = take(es * N);
  L.xib = take(es * (nx + 1));
  L.xisb = take(es * nx);
  L.xfac = take(es * ny);
  L.yib = take(es * (ny + 1));
  L.yisb = take(es * ny);
  L.tanR = take(es * ny);
  L.gidx = take(sizeof(long long) * std::max(p.max_gauges, 1));
  L.gtab = take(sizeof(int) * 3 * (size_t)std::max(p.max_gauges, 1));
  L.grec = take(sizeof(double) * 3 * (size_t)std::max(p.max_gauges, 1) *
                std::max(p.gauge_capacity, 1));
  const size_t mp = std::max(p.max_enclosed_points, 1);
  L.sidx = take(sizeof(long long) * 4 * mp);
  L.swt = take(sizeof(double) * 4 * mp);
  L.sout = take(sizeof(int) * 2 * mp);
  L.srec = take(sizeof(double) * 3 * mp * std::max(p.series_capacity, 1));
  for (int s = 0; s < 4; ++s) {
    const size_t np = s < 2 ? ny : nx;
    const size_t fc = std::max(p.forcing_capacity, 0);
    L.ft[s] = take(sizeof(double) * std::max<size_t>(fc, 1));
    L.fv[s] = take(sizeof(double) * 3 * np * std::max<size_t>(fc, 1));
  }
  L.total = o;
  return L;
}

}  // namespace

struct clf_ctx {
  hipStream_t stream = nullptr;
  int fp32 = 0;
  int nx = 0, ny = 0, coord = 0;
  std::vector<double> x, y, d;
  clf_params p{};
  double dt = 0;
  int ssl_passes = 0;
  double max_cfl = 0, min_f = 0;
  char* ws = nullptr;
  Layout L{};
  GridDesc gd{};
  GridDesc* gd_dev = nullptr;
  StepState* st_dev = nullptr;
  SampleDesc sd{};
  SampleDesc* sd_dev = nullptr;
  ForceDesc fd{};
  ForceDesc* fd_dev = nullptr;
  Tile* tiles_dev = nullptr;
  int ntiles = 0, nblocks = 0, seg = 0;
  int slots = 0;  // step-kernel workgroups resident per XCD (0: unknown)
  bool have_state = false;
  long long n = 0;
  int cur = 0;
  bool rec0 = false;
  int ngauge = 0;
  std::vector<int> gix, giy;        // gauge nodes
  std::vector<Tile> tiles_host;     // the tile list as uploaded (without gauge ranges)
  long long g_first = 0;
  std::vector<Enc> enc;
  int npts = 0, rec_len = 0;
  long long s_first = 0;
  bool forcing = false;
  hipStream_t cap_stream = nullptr;   // capture-only stream (never runs work)
  hipGraphExec_t graph = nullptr;     // graph_steps steps starting from buffer 0
  long long graph_replays = 0;
  // step-kernel timing (kernel_timing): a ring of event pairs, recycled
  // after their elapsed time is added up
  std::vector<hipEvent_t> ev0, ev1;
  std::vector<char> ev_pending;
  long long ev_next = 0;
  double ktime_ms = 0.0;
  long long klaunches = 0;
  // adjoint run (caller-owned workspace)
  char* adj_ws = nullptr;
  int adj_N = 0, adj_K = 0, adj_nck = 0;
  bool adj_ready = false;
  std::string err;
};

namespace {

int fail(clf_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_init_error = buf;
  return code;
}

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(ctx, CLF_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// ----- depth preprocessing: written from dstab / newdw / newdc -----
// Wet depths under the minimum are raised to it; then Jacobi passes (rows,
// then columns) replace any wet node whose deeper line neighbour exceeds
// alpha^2 times its depth: by ((sqrt(d_l) + sqrt(d_r))^2)/4 between two wet
// neighbours, by d_wet/alpha^2 next to the coast.
bool ssl_node(double l, double c, double r, double a2, double* out) {
  if (!(c > 0.0)) return false;
  const double big = l > r ? l : r;
  if (!((big / c) > a2)) return false;
  const bool lw = l > 0.0, rw = r > 0.0;
  if (lw && rw) {
    const double s = std::sqrt(l) + std::sqrt(r);
    *out = (s * s) * 0.25;
    return true;
  }
  if (lw) {
    *out = l / a2;
    return true;
  }
  if (rw) {
    *out = r / a2;
    return true;
  }
  return false;
}

int preprocess_depth(int nx, int ny, std::vector<double>& d, double alpha, double dmin) {
  for (double& v : d)
    if (v > 0.0 && v < dmin) v = dmin;
  const double a2 = alpha * alpha;
  std::vector<double> nxt(d.size());
  for (int pass = 1; pass <= 1000; ++pass) {
    bool moved = false;
    nxt = d;
    if (nx >= 3)
      for (int j = 0; j < ny; ++j) {
        const double* row = d.data() + (size_t)j * nx;
        for (int i = 1; i < nx - 1; ++i) {
          double v;
          if (ssl_node(row[i - 1], row[i], row[i + 1], a2, &v) && v != row[i]) {
            nxt[(size_t)j * nx + i] = v;
            moved = true;
          }
        }
      }
    d.swap(nxt);
    nxt = d;
    if (ny >= 3)
      for (int j = 1; j < ny - 1; ++j)
        for (int i = 0; i < nx; ++i) {
          const size_t k = (size_t)j * nx + i;
          double v;
          if (ssl_node(d[k - nx], d[k], d[k + nx], a2, &v) && v != d[k]) {
            nxt[k] = v;
            moved = true;
          }
        }
    d.swap(nxt);
    if (!moved) return pass;
  }
  return -1;
}

// ----- metric arrays -----
// Along a line with coordinates s and scale q: Delta_k = q (s_{k+1} - s_k),
// with ghost spacings Delta_{-1} = Delta_0 and Delta_{n-1} = Delta_{n-2}.
// ib[k] = 1/Delta_{k-1} (k = 0..n), isb[k] = 1/(Delta_{k-1} + Delta_k).
void line_inverse_spacings(const std::vector<double>& s, double q, std::vector<double>& ib,
                           std::vector<double>& isb) {
  const int n = (int)s.size();
  ib.assign(n + 1, 1.0);
  isb.assign(n, 1.0);
  if (n < 2) return;
  std::vector<double> delta(n + 1);
  for (int k = 1; k < n; ++k) delta[k] = q * (s[k] - s[k - 1]);
  delta[0] = delta[1];
  delta[n] = delta[n - 1];
  for (int k = 0; k <= n; ++k) ib[k] = 1.0 / delta[k];
  for (int k = 0; k < n; ++k) isb[k] = 1.0 / (delta[k] + delta[k + 1]);
}

template <class R>
hipError_t upload(const std::vector<double>& v, void* dst, hipStream_t s) {
  std::vector<R> tmp(v.begin(), v.end());
  hipError_t e = hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

hipError_t upload_any(int fp32, const std::vector<double>& v, void* dst, hipStream_t s) {
  return fp32 ? upload<float>(v, dst, s) : upload<double>(v, dst, s);
}

// Natural tile order: segment rows top to bottom, strips left to right.
// Odd segment rows march in decreasing row order, so that adjacent segment
// rows read their shared halo rows at the same phase of their marches.
void natural_tiles(int grid, int nx, int ny, int seg, std::vector<Tile>& t) {
  const int ns = strips_of(nx);
  const int nsegs = (ny + seg - 1) / seg;
  for (int q = 0; q < nsegs; ++q)
    for (int s = 0; s < ns; ++s) {
      Tile tl{};
      tl.grid = grid | ((q & 1) ? kTileReverse : 0);
      tl.x0 = s * STRIP;
      tl.y0 = q * seg;
      tl.rows = std::min(seg, ny - q * seg);
      t.push_back(tl);
    }
}

// XCD-aware order.  Workgroups are dispatched round-robin over the 8 XCDs
// (workgroup b runs on XCD b % 8), each with its own L2.  The natural list
// is cut into 8 contiguous chunks and chunk x is dealt to the workgroups of
// XCD x, so tiles that share halo rows and columns meet in the same L2.
// Slots past the end of a chunk carry rows = 0 (no work).
constexpr int kXcds = 8;

std::vector<Tile> xcd_order(const std::vector<Tile>& nat, int* nblocks) {
  const int n = (int)nat.size();
  const int per = (n + kXcds - 1) / kXcds;
  const int bper = (per + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;  // blocks per XCD
  std::vector<Tile> out((size_t)bper * kXcds * WAVES_PER_BLOCK);
  for (int b = 0; b < bper * kXcds; ++b) {
    const int x = b % kXcds, j = b / kXcds;
    for (int w = 0; w < WAVES_PER_BLOCK; ++w) {
      const int li = j * WAVES_PER_BLOCK + w;
      const int gi = x * per + li;
      Tile tl{0, 0, 0, 0};
      if (li < per && gi < n) tl = nat[gi];
      out[(size_t)b * WAVES_PER_BLOCK + w] = tl;
    }
  }
  *nblocks = bper * kXcds;
  return out;
}

// Gauges go with the tile whose output region holds them: the tile list
// carries, per tile, a range of the gauge table (row, column, gauge index),
// so that the lane storing a gauge node writes its record on record steps.
int upload_tiles_with_gauges(clf_ctx* c) {
  std::vector<Tile> t = c->tiles_host;
  std::vector<int> tab;
  tab.reserve(3 * c->gix.size());
  for (Tile& tl : t) {
    tl.g0 = (int)(tab.size() / 3);
    tl.gn = 0;
    if (tl.rows <= 0) continue;
    for (size_t g = 0; g < c->gix.size(); ++g) {
      const int ix = c->gix[g], iy = c->giy[g];
      if (ix >= tl.x0 && ix < tl.x0 + STRIP && iy >= tl.y0 && iy < tl.y0 + tl.rows) {
        tab.push_back(iy);
        tab.push_back(ix);
        tab.push_back((int)g);
        tl.gn += 1;
      }
    }
  }
  if (!tab.empty())
    HIPCHK(c, hipMemcpyAsync((void*)c->gd.gtab, tab.data(), tab.size() * sizeof(int),
                             hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->tiles_dev, t.data(), t.size() * sizeof(Tile),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CLF_OK;
}

int upload_tiles(clf_ctx* c, const std::vector<Tile>& t, int nblocks, int seg) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  if ((int)t.size() > c->L.ntiles_max)
    return fail(c, CLF_EINVAL, "segment %d too short for the tile table", seg);
  c->tiles_host = t;
  int rc = upload_tiles_with_gauges(c);
  if (rc) return rc;
  c->ntiles = (int)t.size();
  c->nblocks = nblocks;
  c->seg = seg;
  return CLF_OK;
}

int build_tiles(clf_ctx* c, int seg) {
  std::vector<Tile> nat;
  natural_tiles(0, c->nx, c->ny, seg, nat);
  int nb = 0;
  std::vector<Tile> t = xcd_order(nat, &nb);
  return upload_tiles(c, t, nb, seg);
}

// Workgroups that xcd_order gives each XCD for ntiles tiles.
long long blocks_per_xcd(long long ntiles) {
  const long long per = (ntiles + kXcds - 1) / kXcds;
  return (per + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
}

// Step-kernel workgroups resident at once on one XCD (occupancy of the
// variant times compute units / 8); 0 when unknown.
int resident_per_xcd(int fp32, int order, int gflags) {
  int dev = 0, cus = 0, bpc = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (step_blocks_per_cu(fp32, order, gflags, &bpc) != hipSuccess) return 0;
  return bpc * cus / kXcds;
}

// Round-aligned segment lengths.  A wave walks its segment plus 6 halo rows
// at a rate set by latency more than by issue, so a launch takes about
// (number of workgroup waves) x (segment + 6) row times, and a last, partial
// wave of workgroups costs a whole one.  For k = 1, 2, ... kmax this returns
// the shortest segment whose tile list fills at most k full waves of
// resident workgroups.  tiles(seg) is the tile count for a segment length
// (non-increasing in seg).
template <class F>
std::vector<int> round_segments(F tiles, int slots, int seg_max, int kmax) {
  std::vector<int> out;
  if (slots <= 0) return out;
  seg_max = std::max(seg_max, kMinSeg);
  for (int k = 1; k <= kmax; ++k) {
    const long long cap = (long long)k * slots;
    if (blocks_per_xcd(tiles(seg_max)) > cap) continue;
    int lo = kMinSeg, hi = seg_max;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (blocks_per_xcd(tiles(mid)) <= cap) hi = mid;
      else lo = mid + 1;
    }
    if (!out.empty() && out.back() == lo) break;
    out.push_back(lo);
    if (lo == kMinSeg) break;
  }
  return out;
}

std::vector<int> grid_round_segments(int nx, int ny, int slots, int kmax) {
  const long long strips = strips_of(nx);
  return round_segments([&](int s) { return strips * ((ny + s - 1) / s); }, slots,
                        std::min(4096, ny), kmax);
}

int default_segment(int nx, int ny, int slots) {
  // the fewest full waves of workgroups (one, unless the grid is too large
  // for 4096-row segments)
  std::vector<int> r = grid_round_segments(nx, ny, slots, 64);
  if (!r.empty()) return r.front();
  // occupancy unknown: enough tiles to fill the GPU several times over
  const long long strips = strips_of(nx);
  int seg = 256;
  while (seg > 16 && strips * ((ny + seg - 1) / seg) < 4096) seg /= 2;
  return seg;
}

int step_order_of(int nx, int ny) { return ny == 1 ? ORD_X : (nx == 1 ? ORD_Y : ORD_XY); }

// Autotuner: time the step kernel on this grid for candidate segment
// lengths (rows per wavefront tile) from the lake at rest, keep the fastest.
// Results are cached per (nx, ny, precision, flags) for the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune_cache;

int autotune_segment(clf_ctx* c, int* best_seg) {
  const auto key = std::make_tuple(c->nx, c->ny, c->fp32, c->gd.flags);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *best_seg = it->second;
      return CLF_OK;
    }
  }
  // fixed lengths (every 2 rows where the large grids have their optimum,
  // which moves with the GPU by a few rows) plus the round-aligned ones for
  // up to 4 workgroup waves
  std::vector<int> cands = {16, 20, 24, 26, 28, 30, 32, 34, 36, 40, 48, 56, 64, 96, 128, 192, 256};
  for (int sg : grid_round_segments(c->nx, c->ny, c->slots, 4)) cands.push_back(sg);
  std::sort(cands.begin(), cands.end());
  cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float best = 1e30f;
  int bseg = default_segment(c->nx, c->ny, c->slots);
  const int order = step_order_of(c->nx, c->ny);
  // two rounds over the candidates (the first also warms the clocks); keep
  // each candidate's best time
  std::vector<float> tbest(cands.size(), 1e30f);
  for (int round = 0; round < 2; ++round)
    for (size_t ci = 0; ci < tbest.size(); ++ci) {
      const int seg = cands[ci];
      if (seg > 2 * c->ny && ci > 0) break;
      int rc = build_tiles(c, seg);
      if (rc) return rc;
      const int reps = 10;
      for (int k = 0; k < 3 + reps; ++k) {
        if (k == 3) HIPCHK(c, hipEventRecord(e0, c->stream));
        HIPCHK(c, launch_step(c->fp32, order, c->gd.flags, c->gd_dev, c->tiles_dev, c->ntiles,
                              c->st_dev, c->cur, 1, c->nblocks, c->stream));
        c->cur ^= 1;
      }
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      tbest[ci] = std::min(tbest[ci], ms);
    }
  if (std::getenv("CLF_VERBOSE"))
    for (size_t ci = 0; ci < tbest.size(); ++ci)
      std::fprintf(stderr, "clf autotune %dx%d segment %d: %.4f ms / 10 steps\n", c->nx, c->ny,
                   cands[ci], tbest[ci]);
  for (size_t ci = 0; ci < tbest.size(); ++ci)
    if (tbest[ci] < best) {
      best = tbest[ci];
      bseg = cands[ci];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = bseg;
  }
  *best_seg = bseg;
  return CLF_OK;
}

int check_ready(clf_ctx* c) {
  if (!c) return CLF_EINVAL;
  if (!c->have_state) return fail(c, CLF_ESTATE, "no state: call clf_set_initial first");
  return CLF_OK;
}

int sync_and_check(clf_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  StepState st;
  HIPCHK(c, hipMemcpy(&st, c->st_dev, sizeof st, hipMemcpyDeviceToHost));
  if (st.bad) return fail(c, CLF_ENONFINITE, "state became non-finite");
  return CLF_OK;
}

int push_state(clf_ctx* c) {
  StepState st{};
  HIPCHK(c, hipMemcpyAsync(c->st_dev, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CLF_OK;
}

int push_sampling(clf_ctx* c) {
  c->sd.g_first = c->g_first;
  c->sd.s_first = c->s_first;
  c->sd.ngauge = c->ngauge;
  c->sd.npts = c->npts;
  c->sd.rec_len = c->rec_len;
  HIPCHK(c, hipMemcpyAsync(c->sd_dev, &c->sd, sizeof c->sd, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CLF_OK;
}

long long next_level(long long from, int every) {
  // smallest level >= from that is a multiple of every
  return (from + every - 1) / every * every;
}

long long records_between(long long first, int every, long long lo, long long hi) {
  // number of levels L in [lo, hi] with L >= first and L % every == 0
  lo = std::max(lo, first);
  if (hi < lo) return 0;
  long long a = next_level(lo, every);
  if (a > hi) return 0;
  return (hi - a) / every + 1;
}

}  // namespace

extern "C" {

int clf_node_index(int nx, int ny, int ix, int iy, int64_t* index) {
  if (!index || nx < 1 || ny < 1 || ix < 0 || ix >= nx || iy < 0 || iy >= ny) return CLF_EINVAL;
  // 64-bit arithmetic: grids hold up to 2^32 - 1 nodes
  *index = (int64_t)iy * (int64_t)nx + (int64_t)ix;
  return CLF_OK;
}

void clf_default_params(clf_params* p) {
  std::memset(p, 0, sizeof *p);
  p->precision = CLF_FP64;
  p->h_min = 0.1;
  p->manning_n2 = 0.0;
  p->itopo = 1;
  p->dwall = 0.0;
  p->ssl_alpha = 2.0;
  p->ssl_min_depth = 0.1;
  p->sweep_order = CLF_ORDER_XY;
  p->solver = 2;
  p->earth_radius = 6371000.0;
  p->spherical_metric = 1;
  p->cfl_limit = 1.0;
  p->maxout = 1;
  p->gout = 1;
  p->bndout = 1;
  p->max_gauges = 64;
  p->gauge_capacity = 4096;
  p->max_enclosed = 4;
  p->max_enclosed_points = 4 * 2 * (400 + 400);
  p->series_capacity = 64;
  p->forcing_capacity = 0;
  p->segment = 0;
  p->autotune = 0;
  p->graph_steps = 16;
  p->persistent_blocks = 0;
}

// Field arrays above 4 GiB take the step kernel's 64-bit-address variant
// (the common variants reach a node by a 32-bit byte offset).  Setting the
// environment variable CLF_WIDE_OFFSETS=1 selects it for every grid, so that
// it can be checked on small ones.
static bool wide_offsets(int nx, int ny, int fp32) {
  const long long es = fp32 ? 4 : 8;
  if ((long long)nx * ny * es > (1LL << 32)) return true;
  const char* e = std::getenv("CLF_WIDE_OFFSETS");
  return e && e[0] == '1';
}

// FP32 grids whose fields stream from HBM each step (more than the 256 MiB
// last-level cache holds: h, u, v twice, depth and the maxwave pair) stage
// the rows of the march in LDS; the results are the same bits either way.
// The environment variable CLF_LDS_ROWS, read at init, forces it on (1) or
// off (0) for any FP32 grid, so that both can be checked on small ones.
static bool lds_rows(int nx, int ny, int fp32) {
  if (!fp32) return false;
  const char* e = std::getenv("CLF_LDS_ROWS");
  if (e && (e[0] == '0' || e[0] == '1')) return e[0] == '1';
  return (long long)nx * ny * 9 * 4 > (256LL << 20);
}

static int validate(const clf_grid* g, const clf_params* p, clf_ctx* c);

}  // extern "C"

namespace clf {

void build_metrics(const clf_grid& g, const clf_params& p, GridMetrics& m) {
  const std::vector<double> x(g.x, g.x + g.nx), y(g.y, g.y + g.ny);
  m.xfac.assign(g.ny, 1.0);
  m.tanR.assign(g.ny, 0.0);
  const double deg = kPiD / 180.0;
  if (g.coord == CLF_SPHERICAL) {
    // x spacing in degrees with a per-row factor 1/(R cos(lat) pi/180); y in metres
    const double Rd = p.earth_radius * deg;
    line_inverse_spacings(x, 1.0, m.xib, m.xisb);
    for (int j = 0; j < g.ny; ++j) m.xfac[j] = 1.0 / (Rd * std::cos(y[j] * deg));
    line_inverse_spacings(y, Rd, m.yib, m.yisb);
    if (p.spherical_metric)
      for (int j = 0; j < g.ny; ++j) m.tanR[j] = std::tan(y[j] * deg) / p.earth_radius;
  } else {
    line_inverse_spacings(x, 1.0, m.xib, m.xisb);
    line_inverse_spacings(y, 1.0, m.yib, m.yisb);
  }
}

int grid_flags(const clf_grid& g, const clf_params& p) {
  int flags = 0;
  const int fp32 = p.precision == CLF_FP32;
  if (g.coord == CLF_SPHERICAL && p.spherical_metric) flags |= G_SPHSRC;
  if (p.itopo == 0) flags |= G_WALLMODE;
  if (p.solver == 1) flags |= G_SOLVER1;
  if (p.manning_n2 > 0.0) flags |= G_FRICTION;
  if (p.manning_n2 > 0.0 && p.friction_form == 1) flags |= G_FRIC_SEMI;
  // open edges of a 1-D grid: only the ends along its one dimension matter
  if (p.open_sides & 1) flags |= G_OPEN_W;
  if (p.open_sides & 2) flags |= G_OPEN_E;
  if (p.open_sides & 4) flags |= G_OPEN_S;
  if (p.open_sides & 8) flags |= G_OPEN_N;
  if (wide_offsets(g.nx, g.ny, fp32)) flags |= G_WIDE;
  else if (lds_rows(g.nx, g.ny, fp32)) flags |= G_LDSROWS;
  if (!fp32 && p.h_min < 1e-200) flags |= G_TINYH;
  return flags;
}

void set_step_constants(GridDesc& gd, double dt, const clf_params& p) {
  gd.dt = dt;
  gd.hdt = 0.5 * dt;
  gd.dt2 = dt * dt;
  gd.hmin = p.h_min;
  gd.gn2 = kGrav * p.manning_n2;
  gd.inv16g = 1.0 / (16.0 * kGrav);
  gd.dwall = p.dwall;
}

std::vector<Tile> grid_tiles(int nx, int ny, int seg, int* nblocks) {
  std::vector<Tile> nat;
  natural_tiles(0, nx, ny, seg, nat);
  return xcd_order(nat, nblocks);
}

int grid_default_segment(int nx, int ny, int fp32, int gflags) {
  return default_segment(nx, ny, resident_per_xcd(fp32, step_order_of(nx, ny), gflags));
}

int step_order_for(int nx, int ny) { return step_order_of(nx, ny); }

int validate_args(const clf_grid* g, const clf_params* p) { return validate(g, p, nullptr); }

void set_init_error(const char* msg) { g_init_error = msg; }

}  // namespace clf

extern "C" {

static int validate(const clf_grid* g, const clf_params* p, clf_ctx* c) {
  if (!g || !p) return fail(c, CLF_EINVAL, "null grid or params");
  if (g->nx < 1 || g->ny < 1) return fail(c, CLF_EINVAL, "nx, ny must be >= 1");
  const bool oned = g->nx == 1 || g->ny == 1;
  if (oned && (long long)g->nx * g->ny < 3)
    return fail(c, CLF_EINVAL, "a 1-D grid needs at least 3 nodes");
  if (!oned && (g->nx < 3 || g->ny < 3))
    return fail(c, CLF_EINVAL, "a 2-D grid needs at least 3 nodes per direction");
  if (g->coord != CLF_CARTESIAN && g->coord != CLF_SPHERICAL)
    return fail(c, CLF_EINVAL, "bad coordinate system");
  if (!g->x || !g->y) return fail(c, CLF_EINVAL, "null coordinates");
  for (int i = 0; i + 1 < g->nx; ++i)
    if (!(g->x[i + 1] > g->x[i])) return fail(c, CLF_EINVAL, "x not strictly increasing");
  for (int j = 0; j + 1 < g->ny; ++j)
    if (!(g->y[j + 1] > g->y[j])) return fail(c, CLF_EINVAL, "y not strictly increasing");
  if (g->coord == CLF_SPHERICAL)
    for (int j = 0; j < g->ny; ++j)
      if (!(std::fabs(g->y[j]) < 89.9)) return fail(c, CLF_EINVAL, "latitude out of range");
  if (p->precision != CLF_FP64 && p->precision != CLF_FP32)
    return fail(c, CLF_EINVAL, "bad precision");
  if (p->precision == CLF_FP32 && !kHaveFp32Kernels)
    return fail(c, CLF_EINVAL, "FP32 kernels are not built into this library");
  // node offsets in the step kernel are 32-bit element counts
  if ((long long)g->nx * g->ny >= (1LL << 32))
    return fail(c, CLF_EINVAL, "grid too large: nx * ny must be below 2^32");
  if (!(p->h_min > 0.0)) return fail(c, CLF_EINVAL, "h_min must be > 0");
  if (p->manning_n2 < 0.0) return fail(c, CLF_EINVAL, "manning_n2 must be >= 0");
  if (p->solver != 1 && p->solver != 2) return fail(c, CLF_EINVAL, "solver must be 1 or 2");
  if (p->friction_form != 0 && p->friction_form != 1)
    return fail(c, CLF_EINVAL, "friction_form must be 0 (explicit) or 1 (semi-implicit)");
  if (p->kernel_timing != 0 && p->kernel_timing != 1)
    return fail(c, CLF_EINVAL, "kernel_timing must be 0 or 1");
  if (p->open_sides < 0 || p->open_sides > 15)
    return fail(c, CLF_EINVAL, "open_sides must be a bit mask of the four sides (0..15)");
  if (p->sweep_order != CLF_ORDER_XY && p->sweep_order != CLF_ORDER_ALTERNATE)
    return fail(c, CLF_EINVAL, "bad sweep order");
  if (p->maxout < 1 || p->gout < 1 || p->bndout < 1)
    return fail(c, CLF_EINVAL, "maxout, gout, bndout must be >= 1");
  if (p->ssl_alpha < 0.0 || (p->ssl_alpha > 0.0 && !(p->ssl_alpha > 1.0)))
    return fail(c, CLF_EINVAL, "ssl_alpha must be 0 (off) or > 1");
  if (p->max_gauges < 0 || p->gauge_capacity < 0 || p->max_enclosed < 0 ||
      p->max_enclosed_points < 0 || p->series_capacity < 0 || p->forcing_capacity < 0)
    return fail(c, CLF_EINVAL, "negative capacity");
  if (p->earth_radius <= 0.0) return fail(c, CLF_EINVAL, "earth_radius must be > 0");
  if (p->segment != 0 && (p->segment < kMinSeg || p->segment > 4096))
    return fail(c, CLF_EINVAL, "segment must be 0 (automatic) or in [%d, 4096]", kMinSeg);
  if (p->graph_steps < 0 || (p->graph_steps % 2) != 0 || p->graph_steps > 4096)
    return fail(c, CLF_EINVAL, "graph_steps must be an even number in [0, 4096]");
  if (p->persistent_blocks < 0 || (p->persistent_blocks % 8) != 0)
    return fail(c, CLF_EINVAL, "persistent_blocks must be a non-negative multiple of 8");
  return CLF_OK;
}

int clf_workspace_bytes(const clf_grid* g, const clf_params* p, size_t* bytes) {
  int rc = validate(g, p, nullptr);
  if (rc) return rc;
  if (!bytes) return fail(nullptr, CLF_EINVAL, "null output");
  *bytes = plan(g->nx, g->ny, *p).total;
  return CLF_OK;
}

// Set up one grid context in a workspace region.  with_tiles: build the
// context's own tile list (and autotune); ensemble members skip it.
// Still-water Courant number |lambda| dt / dx over wet nodes (stability
// remark after solver2) and the smallest stability factor f_j (eq:f) of a
// wet node between two wet line neighbours, along both axes.
static void still_water_checks(int nx, int ny, const std::vector<double>& d, double dt,
                               const GridMetrics& M, double* cmax_out, double* fmin_out) {
  double cmax = 0.0, fmin = 1e300;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double dd = d[(size_t)j * nx + i];
      if (!(dd > 0.0)) continue;
      const double cs = std::sqrt(kGrav * dd) * dt;
      if (nx > 1) cmax = std::max(cmax, cs * M.xfac[j] * std::max(M.xib[i], M.xib[i + 1]));
      if (ny > 1) cmax = std::max(cmax, cs * std::max(M.yib[j], M.yib[j + 1]));
      auto fj = [&](double l, double r) {
        if (l > 0.0 && r > 0.0)
          fmin = std::min(fmin, (6.0 * std::sqrt(dd) - std::sqrt(l) - std::sqrt(r)) /
                                    (4.0 * std::sqrt(dd)));
      };
      if (i > 0 && i + 1 < nx) fj(d[(size_t)j * nx + i - 1], d[(size_t)j * nx + i + 1]);
      if (j > 0 && j + 1 < ny) fj(d[(size_t)(j - 1) * nx + i], d[(size_t)(j + 1) * nx + i]);
    }
  *cmax_out = cmax;
  *fmin_out = fmin;
}

static int ctx_create(clf_ctx** out, const clf_grid* g, const double* depth, double dt,
                      const clf_params* p, void* stream, void* ws, size_t ws_bytes,
                      bool with_tiles) {
  if (!out) return fail(nullptr, CLF_EINVAL, "null output");
  *out = nullptr;
  int rc = validate(g, p, nullptr);
  if (rc) return rc;
  if (!depth) return fail(nullptr, CLF_EINVAL, "null depth");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(nullptr, CLF_EINVAL, "dt must be > 0");
  if (!ws) return fail(nullptr, CLF_EINVAL, "null workspace");
  Layout L = plan(g->nx, g->ny, *p);
  if (ws_bytes < L.total)
    return fail(nullptr, CLF_ENOSPACE, "workspace too small: %zu < %zu", ws_bytes, L.total);
  if (((uintptr_t)ws) % 256 != 0) return fail(nullptr, CLF_EINVAL, "workspace not 256-B aligned");

  clf_ctx* c = new clf_ctx();
  c->stream = (hipStream_t)stream;
  c->p = *p;
  c->fp32 = p->precision == CLF_FP32;
  c->nx = g->nx;
  c->ny = g->ny;
  c->coord = g->coord;
  c->x.assign(g->x, g->x + g->nx);
  c->y.assign(g->y, g->y + g->ny);
  const size_t N = (size_t)c->nx * c->ny;
  c->d.assign(depth, depth + N);
  for (size_t k = 0; k < N; ++k)
    if (!std::isfinite(c->d[k])) {
      delete c;
      return fail(nullptr, CLF_EINVAL, "non-finite depth");
    }
  c->dt = dt;
  c->ws = (char*)ws;
  c->L = L;

  if (p->ssl_alpha > 0.0) {
    c->ssl_passes = preprocess_depth(c->nx, c->ny, c->d, p->ssl_alpha, p->ssl_min_depth);
    if (c->ssl_passes < 0) {
      delete c;
      return fail(nullptr, CLF_ESSL, "depth preprocessing did not converge in 1000 passes");
    }
  }

  // metrics
  GridMetrics M;
  build_metrics(*g, *p, M);
  const std::vector<double>&xib = M.xib, &xisb = M.xisb, &yib = M.yib, &yisb = M.yisb,
                            &xfac = M.xfac, &tanR = M.tanR;

  // still-water Courant number over wet nodes, and min f_j (eq:f)
  double cmax = 0.0, fmin = 1e300;
  still_water_checks(c->nx, c->ny, c->d, dt, M, &cmax, &fmin);
  c->max_cfl = cmax;
  c->min_f = fmin;
  if (cmax > p->cfl_limit) {
    delete c;
    return fail(nullptr, CLF_ECFL, "still-water Courant number %.4f exceeds %.4f", cmax,
                p->cfl_limit);
  }

  // carve the workspace
  char* b = c->ws;
  c->gd_dev = (GridDesc*)(b + L.gd);
  c->st_dev = (StepState*)(b + L.st);
  c->sd_dev = (SampleDesc*)(b + L.sd);
  c->fd_dev = (ForceDesc*)(b + L.fd);
  c->tiles_dev = (Tile*)(b + L.tiles);
  GridDesc& gd = c->gd;
  gd.nx = c->nx;
  gd.ny = c->ny;
  gd.flags = grid_flags(*g, *p);
  gd.maxout = p->maxout;
  gd.H[0] = b + L.f[0]; gd.H[1] = b + L.f[1];
  gd.U[0] = b + L.f[2]; gd.U[1] = b + L.f[3];
  gd.V[0] = b + L.f[4]; gd.V[1] = b + L.f[5];
  gd.D = b + L.f[6];
  gd.emax = b + L.f[7];
  gd.smax2 = b + L.f[8];
  gd.xib = b + L.xib;
  gd.xisb = b + L.xisb;
  gd.xfac = b + L.xfac;
  gd.yib = b + L.yib;
  gd.yisb = b + L.yisb;
  gd.tanR = b + L.tanR;
  gd.gtab = (const int*)(b + L.gtab);
  gd.grec = (double*)(b + L.grec);
  gd.ngauge = 0;
  set_step_constants(gd, dt, *p);

  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload_any(c->fp32, c->d, (void*)gd.D, s);
  if (e == hipSuccess) e = upload_any(c->fp32, xib, (void*)gd.xib, s);
  if (e == hipSuccess) e = upload_any(c->fp32, xisb, (void*)gd.xisb, s);
  if (e == hipSuccess) e = upload_any(c->fp32, xfac, (void*)gd.xfac, s);
  if (e == hipSuccess) e = upload_any(c->fp32, yib, (void*)gd.yib, s);
  if (e == hipSuccess) e = upload_any(c->fp32, yisb, (void*)gd.yisb, s);
  if (e == hipSuccess) e = upload_any(c->fp32, tanR, (void*)gd.tanR, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->gd_dev, &gd, sizeof gd, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    std::string m = hipGetErrorString(e);
    delete c;
    return fail(nullptr, CLF_EHIP, "upload failed: %s", m.c_str());
  }

  // sampling and forcing tables
  c->sd = SampleDesc{};
  c->sd.gout = p->gout;
  c->sd.bndout = p->bndout;
  c->sd.gidx = (const long long*)(b + L.gidx);
  c->sd.grec = (double*)(b + L.grec);
  c->sd.gcap = p->gauge_capacity;
  c->sd.sidx = (const long long*)(b + L.sidx);
  c->sd.swt = (const double*)(b + L.swt);
  c->sd.sout = (const int*)(b + L.sout);
  c->sd.srec = (double*)(b + L.srec);
  c->sd.scap = p->series_capacity;
  c->sd.grid = 0;
  c->fd = ForceDesc{};
  c->fd.grid = 0;
  for (int sd = 0; sd < 4; ++sd) {
    c->fd.t[sd] = (const double*)(b + L.ft[sd]);
    c->fd.vals[sd] = (const double*)(b + L.fv[sd]);
  }
  int r2 = push_sampling(c);
  if (r2 == CLF_OK) {
    hipError_t e2 = hipMemcpyAsync(c->fd_dev, &c->fd, sizeof c->fd, hipMemcpyHostToDevice, s);
    if (e2 != hipSuccess) r2 = fail(c, CLF_EHIP, "forcing table upload failed");
  }
  c->slots = resident_per_xcd(c->fp32, step_order_of(c->nx, c->ny), c->gd.flags);
  int seg = p->segment > 0 ? p->segment : default_segment(c->nx, c->ny, c->slots);
  if (r2 == CLF_OK && with_tiles) r2 = build_tiles(c, seg);
  if (r2 == CLF_OK) {
    // lake at rest: h = max(d, 0), dry at or below h_min
    c->have_state = true;
    r2 = clf_set_initial(c, nullptr, nullptr, nullptr, 0);
  }
  if (r2 == CLF_OK && with_tiles && p->autotune && p->segment <= 0) {
    r2 = autotune_segment(c, &seg);
    if (r2 == CLF_OK) r2 = build_tiles(c, seg);
    if (r2 == CLF_OK) r2 = clf_set_initial(c, nullptr, nullptr, nullptr, 0);
  }
  if (r2 != CLF_OK) {
    g_init_error = c->err;
    delete c;
    return r2;
  }
  *out = c;
  return CLF_OK;
}

int clf_init(clf_ctx** out, const clf_grid* g, const double* depth, double dt,
             const clf_params* p, void* stream, void* ws, size_t ws_bytes) {
  TraceRange trace_("clf_init");
  return ctx_create(out, g, depth, dt, p, stream, ws, ws_bytes, true);
}

int clf_set_initial(clf_ctx* c, const double* eta, const double* u, const double* v,
                    int deform_bottom) {
  if (!c) return CLF_EINVAL;
  const long long N = (long long)c->nx * c->ny;
  c->cur = 0;
  HIPCHK(c, launch_init_state(c->fp32, &c->gd, c->gd_dev, eta, u, v, deform_bottom ? 1 : 0, N,
                              c->cur, c->stream));
  HIPCHK(c, launch_clear_maxwave(c->fp32, &c->gd, N, c->stream));
  c->have_state = true;
  c->n = 0;
  c->rec0 = false;
  c->g_first = 0;
  c->s_first = 0;
  int rc = push_state(c);
  return rc ? rc : push_sampling(c);
}

int clf_set_raw_state(clf_ctx* c, const double* h, const double* u, const double* v, int64_t n) {
  if (!c) return CLF_EINVAL;
  if (!h || !u || !v) return fail(c, CLF_EINVAL, "raw state needs h, u and v");
  if (n < 0) return fail(c, CLF_EINVAL, "negative step index");
  const long long N = (long long)c->nx * c->ny;
  c->cur = 0;
  HIPCHK(c, launch_set_raw(c->fp32, &c->gd, c->gd_dev, h, u, v, N, c->cur, c->stream));
  c->have_state = true;
  c->n = n;
  c->rec0 = n > 0;  // the record of level n was taken by the run that reached it
  c->g_first = next_level(c->rec0 ? n + 1 : n, c->p.gout);
  c->s_first = next_level(c->rec0 ? n + 1 : n, c->p.bndout);
  int rc = push_state(c);
  return rc ? rc : push_sampling(c);
}

int clf_get_raw_state(clf_ctx* c, double* h, double* u, double* v) {
  int rc = check_ready(c);
  if (rc) return rc;
  const long long N = (long long)c->nx * c->ny;
  HIPCHK(c, launch_get_raw(c->fp32, &c->gd, c->gd_dev, h, u, v, N, c->cur, c->stream));
  return sync_and_check(c);
}

int clf_set_boundary_forcing(clf_ctx* c, int side, int nt, const double* t, const double* vals) {
  if (!c) return CLF_EINVAL;
  if (side < 0 || side > 3) return fail(c, CLF_EINVAL, "bad side");
  if ((c->nx == 1 && side < 2) || (c->ny == 1 && side >= 2))
    return fail(c, CLF_EINVAL, "side not present on this 1-D grid");
  if (nt < 1 || !t || !vals) return fail(c, CLF_EINVAL, "empty forcing series");
  if (nt > c->p.forcing_capacity)
    return fail(c, CLF_ENOSPACE, "forcing series of %d levels exceeds forcing_capacity %d", nt,
                c->p.forcing_capacity);
  for (int k = 0; k + 1 < nt; ++k)
    if (!(t[k + 1] > t[k])) return fail(c, CLF_EINVAL, "forcing times not increasing");
  const int np = side < 2 ? c->ny : c->nx;
  HIPCHK(c, hipMemcpyAsync((void*)c->fd.t[side], t, sizeof(double) * nt, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync((void*)c->fd.vals[side], vals, sizeof(double) * 3 * np * (size_t)nt,
                           hipMemcpyHostToDevice, c->stream));
  c->fd.nt[side] = nt;
  c->fd.np[side] = np;
  HIPCHK(c, hipMemcpyAsync(c->fd_dev, &c->fd, sizeof c->fd, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int bit[4] = {G_FIX_W, G_FIX_E, G_FIX_S, G_FIX_N};
  c->gd.flags |= bit[side];
  HIPCHK(c, hipMemcpyAsync(c->gd_dev, &c->gd, sizeof c->gd, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->forcing = true;
  return CLF_OK;
}

int clf_set_gauges(clf_ctx* c, int n, const int32_t* ix, const int32_t* iy) {
  if (!c) return CLF_EINVAL;
  if (n < 0 || n > c->p.max_gauges)
    return fail(c, CLF_ENOSPACE, "%d gauges exceed max_gauges %d", n, c->p.max_gauges);
  if (n > 0 && (!ix || !iy)) return fail(c, CLF_EINVAL, "null gauge index");
  std::vector<long long> idx(n);
  for (int g = 0; g < n; ++g) {
    if (ix[g] < 0 || ix[g] >= c->nx || iy[g] < 0 || iy[g] >= c->ny)
      return fail(c, CLF_EINVAL, "gauge %d outside the grid", g);
    int64_t k = 0;
    clf_node_index(c->nx, c->ny, ix[g], iy[g], &k);
    idx[g] = (long long)k;
  }
  if (n > 0)
    HIPCHK(c, hipMemcpyAsync((void*)c->sd.gidx, idx.data(), sizeof(long long) * n,
                             hipMemcpyHostToDevice, c->stream));
  c->ngauge = n;
  c->gix.assign(ix, ix + n);
  c->giy.assign(iy, iy + n);
  c->gd.ngauge = n;
  HIPCHK(c, hipMemcpyAsync(c->gd_dev, &c->gd, sizeof c->gd, hipMemcpyHostToDevice, c->stream));
  if (!c->tiles_host.empty()) {
    int rc = upload_tiles_with_gauges(c);
    if (rc) return rc;
  }
  // records restart at the current level (or at 0 before the first step)
  c->g_first = c->rec0 ? next_level(c->n + 1, c->p.gout) : next_level(c->n, c->p.gout);
  return push_sampling(c);
}

int clf_add_enclosed_grid(clf_ctx* c, int nx, int ny, const double* x, const double* y, int* id) {
  if (!c) return CLF_EINVAL;
  if (c->nx == 1 || c->ny == 1) return fail(c, CLF_EINVAL, "nesting is not enabled for 1-D grids");
  if (nx < 2 || ny < 2 || !x || !y) return fail(c, CLF_EINVAL, "bad enclosed grid");
  if ((int)c->enc.size() >= c->p.max_enclosed)
    return fail(c, CLF_ENOSPACE, "more than max_enclosed enclosed grids");
  const int pts = 2 * (nx + ny);
  if (c->npts + pts > c->p.max_enclosed_points)
    return fail(c, CLF_ENOSPACE, "enclosed boundary points exceed max_enclosed_points");
  auto locate = [](const std::vector<double>& cc, double pnt, int* i0, double* w) -> bool {
    const int n = (int)cc.size();
    if (!(pnt >= cc[0] && pnt <= cc[n - 1])) return false;
    // largest i <= n-2 with cc[i] <= pnt
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (cc[mid] <= pnt) lo = mid;
      else hi = mid;
    }
    *i0 = lo;
    *w = (pnt - cc[lo]) / (cc[lo + 1] - cc[lo]);
    return true;
  };
  std::vector<long long> sidx((size_t)4 * pts);
  std::vector<double> swt((size_t)4 * pts);
  std::vector<int> off(pts), stride(pts);
  Enc E;
  E.nx = nx;
  E.ny = ny;
  int o = c->rec_len, q = 0;
  for (int s = 0; s < 4; ++s) {
    const int np = s < 2 ? ny : nx;
    E.off[s] = o;
    for (int k = 0; k < np; ++k, ++q) {
      double px, py;
      if (s == 0) { px = x[0]; py = y[k]; }
      else if (s == 1) { px = x[nx - 1]; py = y[k]; }
      else if (s == 2) { px = x[k]; py = y[0]; }
      else { px = x[k]; py = y[ny - 1]; }
      int i0, j0;
      double wx, wy;
      if (!locate(c->x, px, &i0, &wx) || !locate(c->y, py, &j0, &wy))
        return fail(c, CLF_EINVAL, "enclosed grid point outside the master grid");
      const long long base = (long long)j0 * c->nx + i0;
      const long long id4[4] = {base, base + 1, base + c->nx, base + c->nx + 1};
      const double w4[4] = {(1.0 - wx) * (1.0 - wy), wx * (1.0 - wy), (1.0 - wx) * wy, wx * wy};
      for (int cc = 0; cc < 4; ++cc) {
        sidx[(size_t)4 * q + cc] = id4[cc];
        swt[(size_t)4 * q + cc] = w4[cc];
      }
      off[q] = o + k;
      stride[q] = np;
    }
    o += 3 * np;
  }
  // all points of all grids live in one table; append this grid's rows
  const int p0 = c->npts;
  HIPCHK(c, hipMemcpyAsync((void*)(c->sd.sidx + (size_t)4 * p0), sidx.data(),
                           sizeof(long long) * sidx.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync((void*)(c->sd.swt + (size_t)4 * p0), swt.data(),
                           sizeof(double) * swt.size(), hipMemcpyHostToDevice, c->stream));
  // sout = [off of all points..., stride of all points...]: rebuild whole table
  std::vector<int> sout_all((size_t)2 * (p0 + pts));
  if (p0 > 0)
    HIPCHK(c, hipMemcpy(sout_all.data(), c->sd.sout, sizeof(int) * 2 * p0, hipMemcpyDeviceToHost));
  std::vector<int> rebuilt((size_t)2 * (p0 + pts));
  for (int i = 0; i < p0; ++i) {
    rebuilt[i] = sout_all[i];
    rebuilt[(size_t)p0 + pts + i] = sout_all[(size_t)p0 + i];
  }
  for (int i = 0; i < pts; ++i) {
    rebuilt[(size_t)p0 + i] = off[i];
    rebuilt[(size_t)2 * p0 + pts + i] = stride[i];
  }
  HIPCHK(c, hipMemcpyAsync((void*)c->sd.sout, rebuilt.data(), sizeof(int) * rebuilt.size(),
                           hipMemcpyHostToDevice, c->stream));
  c->npts += pts;
  c->rec_len = o;
  c->enc.push_back(E);
  c->s_first = c->rec0 ? next_level(c->n + 1, c->p.bndout) : next_level(c->n, c->p.bndout);
  int rc = push_sampling(c);
  if (rc) return rc;
  if (id) *id = (int)c->enc.size() - 1;
  return CLF_OK;
}

static int eff_blocks(int nblocks, int persistent) {
  return (persistent > 0 && persistent < nblocks) ? persistent : nblocks;
}

// Capture graph_steps consecutive steps (buffer 0 -> ... -> buffer 0) into a
// hipGraph on a capture-only stream.  The sequence is valid for any step
// index when it does not depend on it (checked by the caller).
static int build_graph(int fp32, int order, int gflags, const GridDesc* gd, const Tile* tiles,
                       int ntiles, StepState* st, int nblocks, int steps, hipStream_t* cap,
                       hipGraphExec_t* exec, clf_ctx* c) {
  if (!*cap) HIPCHK(c, hipStreamCreateWithFlags(cap, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(*cap, hipStreamCaptureModeThreadLocal));
  int cur = 0;
  hipError_t le = hipSuccess;
  for (int k = 0; k < steps && le == hipSuccess; ++k) {
    le = launch_step(fp32, order, gflags, gd, tiles, ntiles, st, cur, 1, nblocks, *cap);
    cur ^= 1;
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(*cap, &g);
  if (le != hipSuccess) return fail(c, CLF_EHIP, "launch during capture: %s", hipGetErrorString(le));
  if (ee != hipSuccess) return fail(c, CLF_EHIP, "end capture: %s", hipGetErrorString(ee));
  hipError_t ie = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return fail(c, CLF_EHIP, "graph instantiate: %s", hipGetErrorString(ie));
  return CLF_OK;
}

// Records of the level reached (c->n) by the sampling kernel: the
// enclosed-grid series, and the gauges when `gauges` (the first record of a
// run; later gauge records come from the step kernel itself).
static int launch_sampling(clf_ctx* c, bool gauges) {
  const bool g = gauges && c->ngauge > 0 && c->n % c->p.gout == 0 && c->n >= c->g_first;
  const bool e = c->npts > 0 && c->n % c->p.bndout == 0 && c->n >= c->s_first;
  if (!g && !e) return CLF_OK;
  const int nthr = std::max(g ? c->ngauge : 0, e ? c->npts : 0);
  HIPCHK(c, launch_sample(c->fp32, c->gd_dev, c->sd_dev, nthr, c->n, c->cur, g ? 1 : 0,
                          c->stream));
  return CLF_OK;
}

// Gauge record slot that the step reaching level n + 1 writes, or -1.
static int record_slot(const clf_ctx* c) {
  const long long lvl = c->n + 1;
  if (c->ngauge == 0 || lvl % c->p.gout != 0 || lvl < c->g_first) return -1;
  return (int)((lvl - c->g_first) / c->p.gout);
}

constexpr int kTimingRing = 64;

// Add up the elapsed time of the pending event pair in ring slot i.
static int timing_collect(clf_ctx* c, int i) {
  if (!c->ev_pending[i]) return CLF_OK;
  HIPCHK(c, hipEventSynchronize(c->ev1[i]));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0[i], c->ev1[i]));
  c->ktime_ms += ms;
  c->klaunches += 1;
  c->ev_pending[i] = 0;
  return CLF_OK;
}

static int timing_flush(clf_ctx* c) {
  for (int i = 0; i < (int)c->ev_pending.size(); ++i) {
    int rc = timing_collect(c, i);
    if (rc) return rc;
  }
  return CLF_OK;
}

// One step-kernel launch of clf_step, bracketed by an event pair when the
// context times its kernel.
static int timed_step_launch(clf_ctx* c, int order, int do_max, int nb) {
  const int slot = record_slot(c);
  if (!c->p.kernel_timing) {
    HIPCHK(c, launch_step(c->fp32, order, c->gd.flags, c->gd_dev, c->tiles_dev, c->ntiles,
                          c->st_dev, c->cur, do_max, nb, c->stream, slot));
    return CLF_OK;
  }
  if (c->ev0.empty()) {
    c->ev0.resize(kTimingRing);
    c->ev1.resize(kTimingRing);
    c->ev_pending.assign(kTimingRing, 0);
    for (int i = 0; i < kTimingRing; ++i) {
      HIPCHK(c, hipEventCreate(&c->ev0[i]));
      HIPCHK(c, hipEventCreate(&c->ev1[i]));
    }
  }
  const int i = (int)(c->ev_next % kTimingRing);
  int rc = timing_collect(c, i);
  if (rc) return rc;
  HIPCHK(c, hipEventRecord(c->ev0[i], c->stream));
  HIPCHK(c, launch_step(c->fp32, order, c->gd.flags, c->gd_dev, c->tiles_dev, c->ntiles,
                        c->st_dev, c->cur, do_max, nb, c->stream, slot));
  HIPCHK(c, hipEventRecord(c->ev1[i], c->stream));
  c->ev_pending[i] = 1;
  c->ev_next += 1;
  return CLF_OK;
}

static int step_order(clf_ctx* c) {
  if (c->ny == 1) return ORD_X;
  if (c->nx == 1) return ORD_Y;
  if (c->p.sweep_order == CLF_ORDER_ALTERNATE && (c->n % 2) == 1) return ORD_YX;
  return ORD_XY;
}

int clf_step(clf_ctx* c, int nsteps) {
  TraceRange trace_("clf_step");
  int rc = check_ready(c);
  if (rc) return rc;
  if (nsteps < 0) return fail(c, CLF_EINVAL, "negative step count");
  if (nsteps == 0) return CLF_OK;
  // record capacity for levels [first pending, n + nsteps]
  const long long lo = c->rec0 ? c->n + 1 : c->n;
  const long long hi = c->n + nsteps;
  if (c->ngauge > 0) {
    const long long need = records_between(c->g_first, c->p.gout, c->g_first, hi);
    if (need > c->p.gauge_capacity)
      return fail(c, CLF_ENOSPACE, "gauge records would exceed gauge_capacity (%lld > %d)", need,
                  c->p.gauge_capacity);
  }
  if (c->npts > 0) {
    const long long need = records_between(c->s_first, c->p.bndout, c->s_first, hi);
    if (need > c->p.series_capacity)
      return fail(c, CLF_ENOSPACE, "series records would exceed series_capacity (%lld > %d)",
                  need, c->p.series_capacity);
  }
  (void)lo;
  if (!c->rec0) {
    rc = launch_sampling(c, true);
    if (rc) return rc;
    c->rec0 = true;
  }
  const bool graphable = c->p.graph_steps > 0 && !c->forcing && c->ngauge == 0 && c->npts == 0 &&
                         c->p.maxout == 1 && c->p.sweep_order == CLF_ORDER_XY &&
                         !c->p.kernel_timing;
  const int nb = eff_blocks(c->nblocks, c->p.persistent_blocks);
  int k = 0;
  while (k < nsteps) {
    if (graphable && c->cur == 0 && nsteps - k >= c->p.graph_steps) {
      if (!c->graph) {
        rc = build_graph(c->fp32, step_order(c), c->gd.flags, c->gd_dev, c->tiles_dev, c->ntiles,
                         c->st_dev, nb, c->p.graph_steps, &c->cap_stream, &c->graph, c);
        if (rc) return rc;
      }
      HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
      c->graph_replays += 1;
      c->n += c->p.graph_steps;
      k += c->p.graph_steps;
      continue;
    }
    if (c->forcing)
      HIPCHK(c, launch_forcing(c->fp32, c->gd_dev, c->fd_dev, std::max(c->nx, c->ny), c->n,
                               c->cur, c->stream));
    const int do_max = ((c->n + 1) % c->p.maxout) == 0;
    rc = timed_step_launch(c, step_order(c), do_max, nb);
    if (rc) return rc;
    c->cur ^= 1;
    c->n += 1;
    ++k;
    rc = launch_sampling(c, false);
    if (rc) return rc;
  }
  return CLF_OK;
}

int clf_sweep(clf_ctx* c, int axis) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (axis != 0 && axis != 1) return fail(c, CLF_EINVAL, "axis must be 0 or 1");
  if ((axis == 0 && c->nx == 1) || (axis == 1 && c->ny == 1))
    return fail(c, CLF_EINVAL, "no sweep along a dimension of length 1");
  HIPCHK(c, launch_step(c->fp32, axis == 0 ? ORD_X : ORD_Y, c->gd.flags, c->gd_dev, c->tiles_dev, c->ntiles,
                        c->st_dev, c->cur, 0, c->nblocks, c->stream));
  c->cur ^= 1;
  return CLF_OK;
}

int clf_get_state(clf_ctx* c, double* eta, double* u, double* v, uint8_t* wet) {
  int rc = check_ready(c);
  if (rc) return rc;
  const long long N = (long long)c->nx * c->ny;
  HIPCHK(c, launch_get_state(c->fp32, &c->gd, c->gd_dev, eta, u, v, wet, N, c->cur, c->stream));
  return sync_and_check(c);
}

int clf_get_depth(clf_ctx* c, double* d) {
  if (!c || !d) return CLF_EINVAL;
  const long long N = (long long)c->nx * c->ny;
  HIPCHK(c, launch_get_depth(c->fp32, &c->gd, c->gd_dev, d, N, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CLF_OK;
}

int clf_read_gauges(clf_ctx* c, double* out, double* times, int* nrec, int max_rec) {
  int rc = check_ready(c);
  if (rc) return rc;
  rc = sync_and_check(c);
  if (rc) return rc;
  long long have = 0;
  if (c->ngauge > 0 && c->rec0)
    have = records_between(c->g_first, c->p.gout, c->g_first, c->n);
  have = std::min<long long>(have, c->p.gauge_capacity);
  if (nrec) *nrec = (int)have;
  const long long cp = std::min<long long>(have, std::max(max_rec, 0));
  if (cp > 0 && out)
    HIPCHK(c, hipMemcpy(out, c->sd.grec, sizeof(double) * 3 * c->ngauge * cp,
                        hipMemcpyDeviceToHost));
  if (times)
    for (long long r = 0; r < cp; ++r)
      times[r] = (double)(c->g_first + r * c->p.gout) * c->dt;
  return CLF_OK;
}

int clf_read_maxwave(clf_ctx* c, double* eta_max, double* speed_max) {
  int rc = check_ready(c);
  if (rc) return rc;
  const long long N = (long long)c->nx * c->ny;
  HIPCHK(c, launch_read_maxwave(c->fp32, &c->gd, c->gd_dev, eta_max, speed_max, N, c->stream));
  return sync_and_check(c);
}

int clf_read_boundary_series(clf_ctx* c, int id, int side, double* vals, double* times,
                             int* nrec, int max_rec) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (id < 0 || id >= (int)c->enc.size()) return fail(c, CLF_EINVAL, "bad enclosed grid id");
  if (side < 0 || side > 3) return fail(c, CLF_EINVAL, "bad side");
  rc = sync_and_check(c);
  if (rc) return rc;
  long long have = 0;
  if (c->rec0) have = records_between(c->s_first, c->p.bndout, c->s_first, c->n);
  have = std::min<long long>(have, c->p.series_capacity);
  if (nrec) *nrec = (int)have;
  const long long cp = std::min<long long>(have, std::max(max_rec, 0));
  const Enc& E = c->enc[id];
  const int np = side < 2 ? E.ny : E.nx;
  if (cp > 0 && vals) {
    std::vector<double> rec((size_t)c->rec_len);
    for (long long r = 0; r < cp; ++r) {
      HIPCHK(c, hipMemcpy(vals + (size_t)r * 3 * np,
                          c->sd.srec + (size_t)r * c->rec_len + E.off[side],
                          sizeof(double) * 3 * np, hipMemcpyDeviceToHost));
    }
  }
  if (times)
    for (long long r = 0; r < cp; ++r)
      times[r] = (double)(c->s_first + r * c->p.bndout) * c->dt;
  return CLF_OK;
}

int clf_clear_records(clf_ctx* c) {
  if (!c) return CLF_EINVAL;
  const long long from = c->rec0 ? c->n + 1 : c->n;
  c->g_first = next_level(from, c->p.gout);
  c->s_first = next_level(from, c->p.bndout);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return push_sampling(c);
}

int clf_sync(clf_ctx* c) {
  if (!c) return CLF_EINVAL;
  return sync_and_check(c);
}

int clf_query(clf_ctx* c, int what, double* value) {
  if (!c || !value) return CLF_EINVAL;
  switch (what) {
    case CLF_Q_MAX_CFL: *value = c->max_cfl; break;
    case CLF_Q_SSL_PASSES: *value = c->ssl_passes; break;
    case CLF_Q_STEP: *value = (double)c->n; break;
    case CLF_Q_MIN_F: *value = c->min_f; break;
    case CLF_Q_WORKSPACE: *value = (double)c->L.total; break;
    case CLF_Q_GAUGE_RECORDS: {
      long long have = 0;
      if (c->ngauge > 0 && c->rec0) have = records_between(c->g_first, c->p.gout, c->g_first, c->n);
      *value = (double)have;
      break;
    }
    case CLF_Q_TILES: *value = c->ntiles; break;
    case CLF_Q_SEGMENT: *value = c->seg; break;
    case CLF_Q_BLOCKS: *value = eff_blocks(c->nblocks, c->p.persistent_blocks); break;
    case CLF_Q_GRAPH_REPLAYS: *value = (double)c->graph_replays; break;
    case CLF_Q_WIDE: *value = (c->gd.flags & G_WIDE) ? 1.0 : 0.0; break;
    case CLF_Q_LDS_ROWS: *value = (c->gd.flags & G_LDSROWS) ? 1.0 : 0.0; break;
    case CLF_Q_KERNEL_MS:
    case CLF_Q_KERNEL_LAUNCHES:
    case CLF_Q_KERNEL_RESET: {
      int rc = timing_flush(c);
      if (rc) return rc;
      if (what == CLF_Q_KERNEL_MS) *value = c->klaunches ? c->ktime_ms / c->klaunches : 0.0;
      else *value = (double)c->klaunches;
      if (what == CLF_Q_KERNEL_RESET) {
        c->ktime_ms = 0.0;
        c->klaunches = 0;
      }
      break;
    }
    default: return fail(c, CLF_EINVAL, "unknown query %d", what);
  }
  return CLF_OK;
}

const char* clf_last_error(const clf_ctx* c) {
  return c ? c->err.c_str() : g_init_error.c_str();
}

int clf_destroy(clf_ctx* c) {
  if (!c) return CLF_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  for (size_t i = 0; i < c->ev0.size(); ++i) {
    if (c->ev0[i]) (void)hipEventDestroy(c->ev0[i]);
    if (c->ev1[i]) (void)hipEventDestroy(c->ev1[i]);
  }
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return CLF_OK;
}

}  // extern "C"

// ===========================================================================
// Adjoint driver: forward run with checkpoints, reverse run by segments.
// Workspace: checkpoints [nck] + segment store pre[K+1], mid[K] + three
// adjoint states + the record adjoints + 2K sweep descriptors.
// ===========================================================================
namespace {

struct AdjLayout {
  size_t state;  // bytes of one (h, u, v) state
  size_t ck, pre, mid, lam, rec, desc, flags, total;
};

AdjLayout adj_plan(const clf_ctx* c, int N, int K, int nck, int nrec_max) {
  AdjLayout A{};
  const size_t NN = (size_t)c->nx * c->ny;
  A.state = align_up(3 * NN * sizeof(double), 256);
  size_t o = 0;
  A.ck = o; o += (size_t)nck * A.state;
  A.pre = o; o += (size_t)(K + 1) * A.state;
  A.mid = o; o += (size_t)K * A.state;
  A.lam = o; o += 3 * A.state;
  A.rec = o; o = align_up(o + sizeof(double) * 3 * (size_t)std::max(c->ngauge, 1) *
                          (size_t)std::max(nrec_max, 1), 256);
  A.desc = o; o = align_up(o + sizeof(GridDesc) * 2 * (size_t)K, 256);
  A.flags = o; o = align_up(o + (size_t)adjoint_flag_count(c->nx, c->ny), 256);
  A.total = o;
  (void)N;
  return A;
}

int adj_K(int N, int ckpt) {
  if (ckpt > 0) return ckpt;
  int K = (int)std::ceil(std::sqrt((double)std::max(N, 1)));
  return std::max(K, 1);
}

struct St3 {
  double* H;
  double* U;
  double* V;
};

St3 st3(char* base, size_t off, size_t NN) {
  double* p = (double*)(base + off);
  return St3{p, p + NN, p + 2 * NN};
}

int copy_state(clf_ctx* c, St3 dst, const double* H, const double* U, const double* V) {
  const size_t b = sizeof(double) * (size_t)c->nx * c->ny;
  HIPCHK(c, hipMemcpyAsync(dst.H, H, b, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dst.U, U, b, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dst.V, V, b, hipMemcpyDeviceToDevice, c->stream));
  return CLF_OK;
}

int adj_records(const clf_ctx* c, int N) {
  return c->ngauge > 0 ? (int)records_between(0, c->p.gout, 0, N) : 0;
}

}  // namespace

extern "C" {

int clf_adjoint_workspace_bytes(const clf_ctx* c, int nsteps, int ckpt_every, size_t* bytes) {
  if (!c || !bytes || nsteps < 1 || ckpt_every < 0) return CLF_EINVAL;
  const int K = adj_K(nsteps, ckpt_every);
  const int nck = (nsteps + K - 1) / K;
  *bytes = adj_plan(c, nsteps, K, nck, adj_records(c, nsteps)).total;
  return CLF_OK;
}

int clf_adjoint_forward(clf_ctx* c, int nsteps, int ckpt_every, void* ws, size_t ws_bytes) {
  TraceRange trace_("clf_adjoint_forward");
  int rc = check_ready(c);
  if (rc) return rc;
  if (c->fp32) return fail(c, CLF_EINVAL, "the adjoint needs an FP64 context");
  if (c->p.sweep_order != CLF_ORDER_XY) return fail(c, CLF_EINVAL, "the adjoint needs the x-y order");
  if (c->forcing) return fail(c, CLF_EINVAL, "the adjoint does not support boundary forcing");
  if (c->gd.flags & G_OPEN_ANY)
    return fail(c, CLF_EINVAL, "the adjoint does not support open edges");
  if (c->n != 0 || c->rec0) return fail(c, CLF_ESTATE, "call clf_set_initial before the forward run");
  if (nsteps < 1 || ckpt_every < 0 || !ws) return fail(c, CLF_EINVAL, "bad adjoint arguments");
  const int K = adj_K(nsteps, ckpt_every);
  const int nck = (nsteps + K - 1) / K;
  AdjLayout A = adj_plan(c, nsteps, K, nck, adj_records(c, nsteps));
  if (ws_bytes < A.total) return fail(c, CLF_ENOSPACE, "adjoint workspace too small");
  if (((uintptr_t)ws) % 256 != 0) return fail(c, CLF_EINVAL, "adjoint workspace not aligned");
  c->adj_ws = (char*)ws;
  c->adj_N = nsteps;
  c->adj_K = K;
  c->adj_nck = nck;
  c->adj_ready = false;
  const size_t NN = (size_t)c->nx * c->ny;
  for (int m = 0; m < nck; ++m) {
    rc = copy_state(c, st3(c->adj_ws, A.ck + (size_t)m * A.state, NN), (const double*)c->gd.H[c->cur],
                    (const double*)c->gd.U[c->cur], (const double*)c->gd.V[c->cur]);
    if (rc) return rc;
    const int len = std::min(K, nsteps - m * K);
    rc = clf_step(c, len);
    if (rc) return rc;
  }
  // sweep descriptors of the segment store: x maps pre[i] -> mid[i] and y
  // maps mid[i] -> pre[i+1]; a 1-D grid maps pre[i] -> pre[i+1] directly
  std::vector<GridDesc> desc(2 * (size_t)K, c->gd);
  const bool two = c->nx > 1 && c->ny > 1;
  for (int i = 0; i < K; ++i) {
    St3 a = st3(c->adj_ws, A.pre + (size_t)i * A.state, NN);
    St3 b = st3(c->adj_ws, A.mid + (size_t)i * A.state, NN);
    St3 n1 = st3(c->adj_ws, A.pre + (size_t)(i + 1) * A.state, NN);
    GridDesc& dx = desc[2 * (size_t)i];
    GridDesc& dy = desc[2 * (size_t)i + 1];
    const St3 xo = two ? b : n1;
    dx.H[0] = a.H; dx.U[0] = a.U; dx.V[0] = a.V;
    dx.H[1] = xo.H; dx.U[1] = xo.U; dx.V[1] = xo.V;
    dy.H[0] = b.H; dy.U[0] = b.U; dy.V[0] = b.V;
    dy.H[1] = n1.H; dy.U[1] = n1.U; dy.V[1] = n1.V;
  }
  HIPCHK(c, hipMemcpyAsync(c->adj_ws + A.desc, desc.data(), sizeof(GridDesc) * desc.size(),
                           hipMemcpyHostToDevice, c->stream));
  rc = sync_and_check(c);
  if (rc) return rc;
  c->adj_ready = true;
  return CLF_OK;
}

int clf_adjoint_backward(clf_ctx* c, const double* rec_adj, int nrec, double* d_eta0,
                         double* d_u0, double* d_v0) {
  TraceRange trace_("clf_adjoint_backward");
  int rc = check_ready(c);
  if (rc) return rc;
  if (!c->adj_ready) return fail(c, CLF_ESTATE, "no adjoint forward run to reverse");
  const int N = c->adj_N, K = c->adj_K, nck = c->adj_nck;
  if (c->n != N) return fail(c, CLF_ESTATE, "the state moved since the adjoint forward run");
  const int nrec_expect = adj_records(c, N);
  if (nrec != nrec_expect)
    return fail(c, CLF_EINVAL, "expected %d gauge records, got %d", nrec_expect, nrec);
  if (nrec > 0 && !rec_adj) return fail(c, CLF_EINVAL, "null record adjoints");
  AdjLayout A = adj_plan(c, N, K, nck, nrec_expect);
  const size_t NN = (size_t)c->nx * c->ny;
  const size_t fb = sizeof(double) * NN;
  char* w = c->adj_ws;
  double* rdev = (double*)(w + A.rec);
  if (nrec > 0)
    HIPCHK(c, hipMemcpyAsync(rdev, rec_adj, sizeof(double) * 3 * c->ngauge * (size_t)nrec,
                             hipMemcpyHostToDevice, c->stream));
  St3 lam[3] = {st3(w, A.lam, NN), st3(w, A.lam + A.state, NN), st3(w, A.lam + 2 * A.state, NN)};
  int L = 0;  // index of the current adjoint state (the others are overwritten)
  HIPCHK(c, hipMemsetAsync(lam[L].H, 0, 3 * fb, c->stream));
  unsigned char* flags = (unsigned char*)(w + A.flags);
  HIPCHK(c, hipMemsetAsync(flags, 0, (size_t)adjoint_flag_count(c->nx, c->ny), c->stream));
  auto inject = [&](long long level, const double* H) -> int {
    if (c->ngauge == 0 || level % c->p.gout != 0) return CLF_OK;
    const long long r = level / c->p.gout;
    HIPCHK(c, launch_inject(&c->gd, H, c->sd.gidx, c->ngauge, rdev + (size_t)3 * c->ngauge * r,
                            lam[L].H, lam[L].U, lam[L].V, c->stream));
    return CLF_OK;
  };
  rc = inject(N, (const double*)c->gd.H[c->cur]);
  if (rc) return rc;
  const bool two = c->nx > 1 && c->ny > 1;
  const int axis1 = c->ny == 1 ? 0 : 1;  // the only sweep of a 1-D grid
  const GridDesc* dtab = (const GridDesc*)(w + A.desc);
  for (int m = nck - 1; m >= 0; --m) {
    const int start = m * K;
    const int len = std::min(K, N - start);
    St3 ck = st3(w, A.ck + (size_t)m * A.state, NN);
    St3 p0 = st3(w, A.pre, NN);
    HIPCHK(c, hipMemcpyAsync(p0.H, ck.H, 3 * fb, hipMemcpyDeviceToDevice, c->stream));
    for (int i = 0; i < len; ++i) {
      if (two) {
        HIPCHK(c, launch_step(0, ORD_X, c->gd.flags, dtab + 2 * i, c->tiles_dev, c->ntiles,
                              c->st_dev, 0, 0, c->nblocks, c->stream));
        HIPCHK(c, launch_step(0, ORD_Y, c->gd.flags, dtab + 2 * i + 1, c->tiles_dev, c->ntiles,
                              c->st_dev, 0, 0, c->nblocks, c->stream));
      } else {
        HIPCHK(c, launch_step(0, axis1 == 0 ? ORD_X : ORD_Y, c->gd.flags, dtab + 2 * i,
                              c->tiles_dev, c->ntiles, c->st_dev, 0, 0, c->nblocks, c->stream));
      }
    }
    for (int i = len - 1; i >= 0; --i) {
      St3 pre = st3(w, A.pre + (size_t)i * A.state, NN);
      if (two) {
        St3 mid = st3(w, A.mid + (size_t)i * A.state, NN);
        const int Mu = (L + 1) % 3, Nx = (L + 2) % 3;
        HIPCHK(c, launch_adjoint_sweep(&c->gd, 1, mid.H, mid.U, mid.V, lam[L].H, lam[L].U,
                                       lam[L].V, lam[Mu].H, lam[Mu].U, lam[Mu].V, flags, c->stream));
        HIPCHK(c, launch_adjoint_sweep(&c->gd, 0, pre.H, pre.U, pre.V, lam[Mu].H, lam[Mu].U,
                                       lam[Mu].V, lam[Nx].H, lam[Nx].U, lam[Nx].V, flags, c->stream));
        L = Nx;
      } else {
        const int Nx = (L + 1) % 3;
        HIPCHK(c, launch_adjoint_sweep(&c->gd, axis1, pre.H, pre.U, pre.V, lam[L].H, lam[L].U,
                                       lam[L].V, lam[Nx].H, lam[Nx].U, lam[Nx].V, flags, c->stream));
        L = Nx;
      }
      rc = inject(start + i, pre.H);
      if (rc) return rc;
    }
  }
  St3 s0 = st3(w, A.ck, NN);
  HIPCHK(c, launch_initial_adjoint(&c->gd, s0.H, lam[L].H, lam[L].U, lam[L].V, d_eta0, d_u0,
                                   d_v0, (long long)NN, c->stream));
  return sync_and_check(c);
}

}  // extern "C"

// ===========================================================================
// Ensemble of grids: member contexts in one workspace, one combined
// descriptor table and tile list, one step-kernel launch per time step.
// ===========================================================================
struct clf_ens {
  hipStream_t stream = nullptr;
  clf_params p{};
  int fp32 = 0;
  int gflags = 0;  // union of the members' flags (kernel variant)
  std::vector<clf_ctx*> m;
  GridDesc* gd_dev = nullptr;
  StepState* st_dev = nullptr;
  Tile* tiles_dev = nullptr;
  int tiles_cap = 0;
  int ntiles = 0, nblocks = 0, seg = 0;
  int slots = 0;  // step-kernel workgroups resident per XCD (0: unknown)
  long long n = 0;
  int cur = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  long long graph_replays = 0;
  std::string err;
};

namespace {

thread_local std::string g_ens_error;

int efail(clf_ens* e, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (e) e->err = buf;
  else g_ens_error = buf;
  return code;
}

#define EHIPCHK(ens, call)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return efail(ens, CLF_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

clf_params member_params(const clf_params& p) {
  clf_params q = p;
  q.max_gauges = 0;
  q.gauge_capacity = 0;
  q.max_enclosed = 0;
  q.max_enclosed_points = 0;
  q.series_capacity = 0;
  q.forcing_capacity = 0;
  q.autotune = 0;
  return q;
}

struct EnsPlan {
  size_t gd, st, tiles, total;
  int tiles_cap;
  std::vector<size_t> off, size;
};

EnsPlan ens_plan(int n, const clf_grid* grids, const clf_params& p) {
  EnsPlan E;
  const clf_params q = member_params(p);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  E.gd = take(sizeof(GridDesc) * (size_t)n);
  E.st = take(sizeof(StepState));
  long long cap = 8LL * WAVES_PER_BLOCK * 2;
  for (int i = 0; i < n; ++i)
    cap += (long long)strips_of(grids[i].nx) * ((grids[i].ny + kMinSeg - 1) / kMinSeg);
  E.tiles_cap = (int)cap;
  E.tiles = take(sizeof(Tile) * (size_t)cap);
  for (int i = 0; i < n; ++i) {
    const size_t sz = plan(grids[i].nx, grids[i].ny, q).total;
    E.off.push_back(take(sz));
    E.size.push_back(sz);
  }
  E.total = o;
  return E;
}

int ens_build_tiles(clf_ens* e, int seg) {
  std::vector<Tile> nat;
  for (size_t i = 0; i < e->m.size(); ++i) natural_tiles((int)i, e->m[i]->nx, e->m[i]->ny, seg, nat);
  int nb = 0;
  std::vector<Tile> t = xcd_order(nat, &nb);
  if ((int)t.size() > e->tiles_cap) return efail(e, CLF_EINVAL, "segment %d too short", seg);
  if (e->graph) {
    (void)hipGraphExecDestroy(e->graph);
    e->graph = nullptr;
  }
  EHIPCHK(e, hipMemcpyAsync(e->tiles_dev, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice,
                            e->stream));
  EHIPCHK(e, hipStreamSynchronize(e->stream));
  e->ntiles = (int)t.size();
  e->nblocks = nb;
  e->seg = seg;
  return CLF_OK;
}

std::vector<int> ens_round_segments(const clf_ens* e, int kmax) {
  int ny_max = 0;
  for (auto* c : e->m) ny_max = std::max(ny_max, c->ny);
  auto tiles = [&](int s) {
    long long t = 0;
    for (auto* c : e->m) t += (long long)strips_of(c->nx) * ((c->ny + s - 1) / s);
    return t;
  };
  return round_segments(tiles, e->slots, std::min(4096, ny_max), kmax);
}

int ens_default_segment(const clf_ens* e) {
  std::vector<int> r = ens_round_segments(e, 64);
  if (!r.empty()) return r.front();
  long long tiles64 = 0;
  for (auto* c : e->m) tiles64 += (long long)strips_of(c->nx) * ((c->ny + 63) / 64);
  return tiles64 >= 4096 ? 64 : 32;
}

int ens_autotune(clf_ens* e, int* best) {
  std::vector<int> cands = {16, 20, 24, 26, 28, 30, 32, 34, 36, 40, 48, 64, 96, 128};
  for (int sg : ens_round_segments(e, 4)) cands.push_back(sg);
  std::sort(cands.begin(), cands.end());
  cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
  hipEvent_t a, b;
  EHIPCHK(e, hipEventCreate(&a));
  EHIPCHK(e, hipEventCreate(&b));
  float tb = 1e30f;
  int bs = ens_default_segment(e);
  for (int round = 0; round < 2; ++round)
    for (int seg : cands) {
      int rc = ens_build_tiles(e, seg);
      if (rc) return rc;
      const int nb = eff_blocks(e->nblocks, e->p.persistent_blocks);
      for (int k = 0; k < 8; ++k) {
        if (k == 2) EHIPCHK(e, hipEventRecord(a, e->stream));
        EHIPCHK(e, launch_step(e->fp32, ORD_XY, e->gflags, e->gd_dev, e->tiles_dev, e->ntiles,
                               e->st_dev, e->cur, 1, nb, e->stream));
        e->cur ^= 1;
      }
      EHIPCHK(e, hipEventRecord(b, e->stream));
      EHIPCHK(e, hipEventSynchronize(b));
      float ms = 0.f;
      EHIPCHK(e, hipEventElapsedTime(&ms, a, b));
      if (round == 1 && ms < tb) {
        tb = ms;
        bs = seg;
      }
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *best = bs;
  return CLF_OK;
}

}  // namespace

extern "C" {

int clf_ensemble_workspace_bytes(int n, const clf_grid* grids, const clf_params* p,
                                 size_t* bytes) {
  if (n < 1 || !grids || !p || !bytes) return efail(nullptr, CLF_EINVAL, "bad arguments");
  for (int i = 0; i < n; ++i) {
    int rc = validate(&grids[i], p, nullptr);
    if (rc) return rc;
  }
  *bytes = ens_plan(n, grids, *p).total;
  return CLF_OK;
}

int clf_ensemble_init(clf_ens** out, int n, const clf_grid* grids, const double* const* depths,
                      const double* dts, const clf_params* p, void* stream, void* ws,
                      size_t ws_bytes) {
  if (!out) return efail(nullptr, CLF_EINVAL, "null output");
  *out = nullptr;
  if (n < 1 || !grids || !depths || !dts || !p || !ws)
    return efail(nullptr, CLF_EINVAL, "bad arguments");
  for (int i = 0; i < n; ++i) {
    int rc = validate(&grids[i], p, nullptr);
    if (rc) return efail(nullptr, rc, "member %d: %s", i, g_init_error.c_str());
    if (grids[i].nx == 1 || grids[i].ny == 1)
      return efail(nullptr, CLF_EINVAL, "member %d: ensemble members must be 2-D", i);
  }
  if (p->sweep_order != CLF_ORDER_XY)
    return efail(nullptr, CLF_EINVAL, "ensembles use the x-y order");
  EnsPlan E = ens_plan(n, grids, *p);
  if (ws_bytes < E.total)
    return efail(nullptr, CLF_ENOSPACE, "workspace too small: %zu < %zu", ws_bytes, E.total);
  if (((uintptr_t)ws) % 256 != 0) return efail(nullptr, CLF_EINVAL, "workspace not aligned");
  clf_ens* e = new clf_ens();
  e->stream = (hipStream_t)stream;
  e->p = *p;
  e->fp32 = p->precision == CLF_FP32;
  char* b = (char*)ws;
  e->gd_dev = (GridDesc*)(b + E.gd);
  e->st_dev = (StepState*)(b + E.st);
  e->tiles_dev = (Tile*)(b + E.tiles);
  e->tiles_cap = E.tiles_cap;
  const clf_params q = member_params(*p);
  std::vector<GridDesc> table;
  for (int i = 0; i < n; ++i) {
    clf_ctx* c = nullptr;
    int rc = ctx_create(&c, &grids[i], depths[i], dts[i], &q, stream, b + E.off[i], E.size[i],
                        false);
    if (rc) {
      std::string msg = g_init_error;
      clf_ensemble_destroy(e);
      return efail(nullptr, rc, "member %d: %s", i, msg.c_str());
    }
    e->m.push_back(c);
    table.push_back(c->gd);
    e->gflags |= c->gd.flags;
  }
  int rc = CLF_OK;
  hipError_t he = hipMemcpyAsync(e->gd_dev, table.data(), sizeof(GridDesc) * n,
                                 hipMemcpyHostToDevice, e->stream);
  StepState st{};
  if (he == hipSuccess)
    he = hipMemcpyAsync(e->st_dev, &st, sizeof st, hipMemcpyHostToDevice, e->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
  if (he != hipSuccess) rc = efail(e, CLF_EHIP, "upload: %s", hipGetErrorString(he));
  e->slots = resident_per_xcd(e->fp32, ORD_XY, e->gflags);
  int seg = p->segment > 0 ? p->segment : ens_default_segment(e);
  if (rc == CLF_OK) rc = ens_build_tiles(e, seg);
  if (rc == CLF_OK && p->autotune && p->segment <= 0) {
    rc = ens_autotune(e, &seg);
    if (rc == CLF_OK) rc = ens_build_tiles(e, seg);
    // back to the lake at rest for every member
    e->cur = 0;
    for (int i = 0; i < n && rc == CLF_OK; ++i)
      rc = clf_ensemble_set_initial(e, i, nullptr, nullptr, nullptr, 0);
  }
  if (rc != CLF_OK) {
    std::string msg = e->err;
    clf_ensemble_destroy(e);
    return efail(nullptr, rc, "%s", msg.c_str());
  }
  *out = e;
  return CLF_OK;
}

int clf_ensemble_set_initial(clf_ens* e, int member, const double* eta, const double* u,
                             const double* v, int deform_bottom) {
  if (!e) return CLF_EINVAL;
  if (member < 0 || member >= (int)e->m.size()) return efail(e, CLF_EINVAL, "bad member");
  clf_ctx* c = e->m[member];
  const long long N = (long long)c->nx * c->ny;
  EHIPCHK(e, launch_init_state(e->fp32, &c->gd, c->gd_dev, eta, u, v, deform_bottom ? 1 : 0, N,
                               e->cur, e->stream));
  EHIPCHK(e, launch_clear_maxwave(e->fp32, &c->gd, N, e->stream));
  if (deform_bottom) {
    // the depth changed on the device; the descriptor (pointers) did not
  }
  return CLF_OK;
}

int clf_ensemble_step(clf_ens* e, int nsteps) {
  TraceRange trace_("clf_ensemble_step");
  if (!e) return CLF_EINVAL;
  if (nsteps < 0) return efail(e, CLF_EINVAL, "negative step count");
  const int nb = eff_blocks(e->nblocks, e->p.persistent_blocks);
  const bool graphable = e->p.graph_steps > 0 && e->p.maxout == 1;
  int k = 0;
  while (k < nsteps) {
    if (graphable && e->cur == 0 && nsteps - k >= e->p.graph_steps) {
      if (!e->graph) {
        clf_ctx tmp;  // error sink for the shared capture helper
        int rc = build_graph(e->fp32, ORD_XY, e->gflags, e->gd_dev, e->tiles_dev, e->ntiles,
                             e->st_dev, nb, e->p.graph_steps, &e->cap_stream, &e->graph, &tmp);
        if (rc) return efail(e, rc, "%s", tmp.err.c_str());
      }
      EHIPCHK(e, hipGraphLaunch(e->graph, e->stream));
      e->graph_replays += 1;
      e->n += e->p.graph_steps;
      k += e->p.graph_steps;
      continue;
    }
    const int do_max = ((e->n + 1) % e->p.maxout) == 0;
    EHIPCHK(e, launch_step(e->fp32, ORD_XY, e->gflags, e->gd_dev, e->tiles_dev, e->ntiles,
                           e->st_dev, e->cur, do_max, nb, e->stream));
    e->cur ^= 1;
    e->n += 1;
    ++k;
  }
  return CLF_OK;
}

int clf_ensemble_sync(clf_ens* e) {
  if (!e) return CLF_EINVAL;
  EHIPCHK(e, hipStreamSynchronize(e->stream));
  StepState st;
  EHIPCHK(e, hipMemcpy(&st, e->st_dev, sizeof st, hipMemcpyDeviceToHost));
  if (st.bad) return efail(e, CLF_ENONFINITE, "state became non-finite");
  return CLF_OK;
}

int clf_ensemble_get_state(clf_ens* e, int member, double* eta, double* u, double* v,
                           uint8_t* wet) {
  if (!e) return CLF_EINVAL;
  if (member < 0 || member >= (int)e->m.size()) return efail(e, CLF_EINVAL, "bad member");
  clf_ctx* c = e->m[member];
  const long long N = (long long)c->nx * c->ny;
  EHIPCHK(e, launch_get_state(e->fp32, &c->gd, c->gd_dev, eta, u, v, wet, N, e->cur, e->stream));
  return clf_ensemble_sync(e);
}

int clf_ensemble_read_maxwave(clf_ens* e, int member, double* eta_max, double* speed_max) {
  if (!e) return CLF_EINVAL;
  if (member < 0 || member >= (int)e->m.size()) return efail(e, CLF_EINVAL, "bad member");
  clf_ctx* c = e->m[member];
  const long long N = (long long)c->nx * c->ny;
  EHIPCHK(e, launch_read_maxwave(e->fp32, &c->gd, c->gd_dev, eta_max, speed_max, N, e->stream));
  return clf_ensemble_sync(e);
}

int clf_ensemble_query(clf_ens* e, int what, double* value) {
  if (!e || !value) return CLF_EINVAL;
  switch (what) {
    case CLF_Q_STEP: *value = (double)e->n; break;
    case CLF_Q_TILES: *value = e->ntiles; break;
    case CLF_Q_SEGMENT: *value = e->seg; break;
    case CLF_Q_BLOCKS: *value = eff_blocks(e->nblocks, e->p.persistent_blocks); break;
    case CLF_Q_GRAPH_REPLAYS: *value = (double)e->graph_replays; break;
    case CLF_Q_WIDE: *value = (e->gflags & G_WIDE) ? 1.0 : 0.0; break;
    case CLF_Q_LDS_ROWS: *value = (e->gflags & G_LDSROWS) ? 1.0 : 0.0; break;
    case CLF_Q_WORKSPACE: {
      double tot = 0;
      for (auto* c : e->m) tot += (double)c->L.total;
      *value = tot;
      break;
    }
    default: return efail(e, CLF_EINVAL, "unknown query %d", what);
  }
  return CLF_OK;
}

const char* clf_ensemble_last_error(const clf_ens* e) {
  return e ? e->err.c_str() : g_ens_error.c_str();
}

int clf_ensemble_destroy(clf_ens* e) {
  if (!e) return CLF_EINVAL;
  (void)hipStreamSynchronize(e->stream);
  if (e->graph) (void)hipGraphExecDestroy(e->graph);
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  for (auto* c : e->m) clf_destroy(c);
  delete e;
  return CLF_OK;
}

}  // extern "C"

// ===========================================================================
// One grid split into y-bands on one device: the per-GPU part of the y-band
// sharding of a large grid.  Each band is an ensemble member holding its own
// rows plus HALO rows beyond each inner edge.  One step is one step-kernel
// launch over every band's tiles followed by one exchange launch: the HALO
// rows beyond each inner edge take the post-step values of the band that owns
// them.  A node's update depends on the pre-step state within HALO rows
// (steps (a)-(e) of the y-sweep reach 3 nodes; the x-sweep is row-local), so
// the owned rows of every band are exactly the whole-grid run's, and after
// the exchange so are the halo rows.
// ===========================================================================
struct clf_bands {
  clf_ens* e = nullptr;
  hipStream_t stream = nullptr;
  int nx = 0, ny = 0, fp32 = 0;
  std::vector<int> r0, r1, g0;  // owned rows [r0, r1); first row of the band's grid g0
  BandXchg* xt_dev = nullptr;
  int nxchg = 0;
  int ssl_passes = 0;
  double max_cfl = 0, min_f = 0;
  std::string err;
};

namespace {

thread_local std::string g_band_error;

int bfail(clf_bands* b, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  else g_band_error = buf;
  return code;
}

struct BandPlan {
  std::vector<int> r0, r1, g0, g1;
  std::vector<std::vector<double>> ys;
  std::vector<clf_grid> grids;
  EnsPlan E;
  size_t xt = 0, total = 0;
};

clf_params band_member_params(const clf_params& p) {
  clf_params q = p;
  q.ssl_alpha = 0.0;     // the whole grid's depth is preprocessed once
  q.cfl_limit = 1e300;   // and checked once, on the whole grid
  return q;
}

int band_plan(const clf_grid* g, const clf_params* p, int nb, BandPlan& P) {
  int rc = validate(g, p, nullptr);
  if (rc) return bfail(nullptr, rc, "%s", g_init_error.c_str());
  if (g->nx < 3 || g->ny < 3) return bfail(nullptr, CLF_EINVAL, "bands need a 2-D grid");
  if (p->sweep_order != CLF_ORDER_XY) return bfail(nullptr, CLF_EINVAL, "bands use the x-y order");
  if (nb < 1 || g->ny / nb < HALO)
    return bfail(nullptr, CLF_EINVAL, "%d bands of %d rows: every band needs %d rows or more", nb,
                 g->ny, HALO);
  const int base = g->ny / nb, extra = g->ny % nb;
  int r = 0;
  for (int b = 0; b < nb; ++b) {
    const int rows = base + (b < extra ? 1 : 0);
    P.r0.push_back(r);
    P.r1.push_back(r + rows);
    P.g0.push_back(std::max(0, r - HALO));
    P.g1.push_back(std::min(g->ny, r + rows + HALO));
    r += rows;
  }
  for (int b = 0; b < nb; ++b) P.ys.emplace_back(g->y + P.g0[b], g->y + P.g1[b]);
  for (int b = 0; b < nb; ++b)
    P.grids.push_back(clf_grid{g->nx, P.g1[b] - P.g0[b], g->coord, g->x, P.ys[b].data()});
  P.E = ens_plan(nb, P.grids.data(), band_member_params(*p));
  P.xt = align_up(P.E.total, 256);
  P.total = align_up(P.xt + sizeof(BandXchg) * 2 * (size_t)nb, 256);
  return CLF_OK;
}

}  // namespace

extern "C" {

int clf_bands_workspace_bytes(const clf_grid* g, const clf_params* p, int nbands, size_t* bytes) {
  if (!g || !p || !bytes) return bfail(nullptr, CLF_EINVAL, "null argument");
  BandPlan P;
  int rc = band_plan(g, p, nbands, P);
  if (rc) return rc;
  *bytes = P.total;
  return CLF_OK;
}

int clf_bands_init(clf_bands** out, const clf_grid* g, const double* depth, double dt,
                   const clf_params* p, int nbands, void* stream, void* ws, size_t ws_bytes) {
  TraceRange trace_("clf_bands_init");
  if (!out) return bfail(nullptr, CLF_EINVAL, "null output");
  *out = nullptr;
  if (!g || !p || !depth || !ws) return bfail(nullptr, CLF_EINVAL, "null argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return bfail(nullptr, CLF_EINVAL, "dt must be > 0");
  BandPlan P;
  int rc = band_plan(g, p, nbands, P);
  if (rc) return rc;
  if (ws_bytes < P.total)
    return bfail(nullptr, CLF_ENOSPACE, "workspace too small: %zu < %zu", ws_bytes, P.total);
  if (((uintptr_t)ws) % 256 != 0) return bfail(nullptr, CLF_EINVAL, "workspace not aligned");
  const size_t N = (size_t)g->nx * g->ny;
  std::vector<double> d(depth, depth + N);
  for (double v : d)
    if (!std::isfinite(v)) return bfail(nullptr, CLF_EINVAL, "non-finite depth");
  int passes = 0;
  if (p->ssl_alpha > 0.0) {
    passes = preprocess_depth(g->nx, g->ny, d, p->ssl_alpha, p->ssl_min_depth);
    if (passes < 0)
      return bfail(nullptr, CLF_ESSL, "depth preprocessing did not converge in 1000 passes");
  }
  GridMetrics M;
  build_metrics(*g, *p, M);
  double cmax = 0.0, fmin = 1e300;
  still_water_checks(g->nx, g->ny, d, dt, M, &cmax, &fmin);
  if (cmax > p->cfl_limit)
    return bfail(nullptr, CLF_ECFL, "still-water Courant number %.4f exceeds %.4f", cmax,
                 p->cfl_limit);
  std::vector<const double*> depths;
  std::vector<double> dts(nbands, dt);
  for (int b = 0; b < nbands; ++b) depths.push_back(d.data() + (size_t)P.g0[b] * g->nx);
  const clf_params q = band_member_params(*p);
  clf_ens* e = nullptr;
  rc = clf_ensemble_init(&e, nbands, P.grids.data(), depths.data(), dts.data(), &q, stream, ws,
                         P.E.total);
  if (rc) return bfail(nullptr, rc, "%s", g_ens_error.c_str());
  clf_bands* bd = new clf_bands();
  bd->e = e;
  bd->stream = (hipStream_t)stream;
  bd->nx = g->nx;
  bd->ny = g->ny;
  bd->fp32 = e->fp32;
  bd->r0 = P.r0;
  bd->r1 = P.r1;
  bd->g0 = P.g0;
  bd->ssl_passes = passes;
  bd->max_cfl = cmax;
  bd->min_f = fmin;
  // each inner edge: the lower band's last HALO owned rows become the upper
  // band's first (halo) rows, and the upper band's first HALO owned rows the
  // lower band's last (halo) rows
  std::vector<BandXchg> xt;
  for (int b = 0; b + 1 < nbands; ++b) {
    const int edge = P.r1[b];
    xt.push_back(BandXchg{b, edge - HALO - P.g0[b], b + 1, edge - HALO - P.g0[b + 1]});
    xt.push_back(BandXchg{b + 1, edge - P.g0[b + 1], b, edge - P.g0[b]});
  }
  bd->nxchg = (int)xt.size();
  bd->xt_dev = (BandXchg*)((char*)ws + P.xt);
  hipError_t he = hipSuccess;
  if (!xt.empty())
    he = hipMemcpyAsync(bd->xt_dev, xt.data(), xt.size() * sizeof(BandXchg),
                        hipMemcpyHostToDevice, bd->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(bd->stream);
  if (he != hipSuccess) {
    clf_bands_destroy(bd);
    return bfail(nullptr, CLF_EHIP, "exchange table upload: %s", hipGetErrorString(he));
  }
  *out = bd;
  return CLF_OK;
}

int clf_bands_set_initial(clf_bands* b, const double* eta, const double* u, const double* v,
                          int deform_bottom) {
  if (!b) return CLF_EINVAL;
  const size_t nx = b->nx;
  for (int k = 0; k < (int)b->r0.size(); ++k) {
    const size_t off = (size_t)b->g0[k] * nx;
    int rc = clf_ensemble_set_initial(b->e, k, eta ? eta + off : nullptr, u ? u + off : nullptr,
                                      v ? v + off : nullptr, deform_bottom);
    if (rc) return bfail(b, rc, "%s", b->e->err.c_str());
  }
  b->e->n = 0;
  return CLF_OK;
}

int clf_bands_step(clf_bands* b, int nsteps) {
  TraceRange trace_("clf_bands_step");
  if (!b) return CLF_EINVAL;
  if (nsteps < 0) return bfail(b, CLF_EINVAL, "negative step count");
  clf_ens* e = b->e;
  const int nb = eff_blocks(e->nblocks, e->p.persistent_blocks);
  for (int k = 0; k < nsteps; ++k) {
    const int do_max = ((e->n + 1) % e->p.maxout) == 0;
    hipError_t he = launch_step(e->fp32, ORD_XY, e->gflags, e->gd_dev, e->tiles_dev, e->ntiles,
                                e->st_dev, e->cur, do_max, nb, b->stream);
    e->cur ^= 1;
    e->n += 1;
    if (he == hipSuccess)
      he = launch_band_exchange(e->fp32, e->gd_dev, b->xt_dev, b->nxchg, b->nx, e->cur, b->stream);
    if (he != hipSuccess) return bfail(b, CLF_EHIP, "band step: %s", hipGetErrorString(he));
  }
  return CLF_OK;
}

int clf_bands_sync(clf_bands* b) {
  if (!b) return CLF_EINVAL;
  int rc = clf_ensemble_sync(b->e);
  return rc ? bfail(b, rc, "%s", b->e->err.c_str()) : CLF_OK;
}

// The owned rows of band k as a grid descriptor of their own (field pointers
// advanced to the first owned row).
static GridDesc owned_rows(const clf_bands* b, int k, long long* N) {
  const clf_ctx* c = b->e->m[k];
  GridDesc gd = c->gd;
  const size_t es = b->fp32 ? 4 : 8;
  const size_t off = (size_t)(b->r0[k] - b->g0[k]) * b->nx * es;
  auto adv = [&](void* ptr) { return (void*)((char*)ptr + off); };
  for (int q = 0; q < 2; ++q) {
    gd.H[q] = adv(gd.H[q]);
    gd.U[q] = adv(gd.U[q]);
    gd.V[q] = adv(gd.V[q]);
  }
  gd.D = adv(gd.D);
  gd.emax = adv(gd.emax);
  gd.smax2 = adv(gd.smax2);
  *N = (long long)(b->r1[k] - b->r0[k]) * b->nx;
  return gd;
}

int clf_bands_get_state(clf_bands* b, double* eta, double* u, double* v, uint8_t* wet) {
  if (!b) return CLF_EINVAL;
  for (int k = 0; k < (int)b->r0.size(); ++k) {
    long long N = 0;
    const GridDesc gd = owned_rows(b, k, &N);
    const size_t o = (size_t)b->r0[k] * b->nx;
    hipError_t he = launch_get_state(b->fp32, &gd, nullptr, eta ? eta + o : nullptr,
                                     u ? u + o : nullptr, v ? v + o : nullptr,
                                     wet ? wet + o : nullptr, N, b->e->cur, b->stream);
    if (he != hipSuccess) return bfail(b, CLF_EHIP, "get state: %s", hipGetErrorString(he));
  }
  return clf_bands_sync(b);
}

int clf_bands_read_maxwave(clf_bands* b, double* eta_max, double* speed_max) {
  if (!b) return CLF_EINVAL;
  for (int k = 0; k < (int)b->r0.size(); ++k) {
    long long N = 0;
    const GridDesc gd = owned_rows(b, k, &N);
    const size_t o = (size_t)b->r0[k] * b->nx;
    hipError_t he = launch_read_maxwave(b->fp32, &gd, nullptr, eta_max ? eta_max + o : nullptr,
                                        speed_max ? speed_max + o : nullptr, N, b->stream);
    if (he != hipSuccess) return bfail(b, CLF_EHIP, "read maxwave: %s", hipGetErrorString(he));
  }
  return clf_bands_sync(b);
}

int clf_bands_query(clf_bands* b, int what, double* value) {
  if (!b || !value) return CLF_EINVAL;
  switch (what) {
    case CLF_Q_MAX_CFL: *value = b->max_cfl; return CLF_OK;
    case CLF_Q_MIN_F: *value = b->min_f; return CLF_OK;
    case CLF_Q_SSL_PASSES: *value = b->ssl_passes; return CLF_OK;
    default: {
      int rc = clf_ensemble_query(b->e, what, value);
      return rc ? bfail(b, rc, "%s", b->e->err.c_str()) : CLF_OK;
    }
  }
}

const char* clf_bands_last_error(const clf_bands* b) {
  return b ? b->err.c_str() : g_band_error.c_str();
}

int clf_bands_destroy(clf_bands* b) {
  if (!b) return CLF_EINVAL;
  if (b->e) clf_ensemble_destroy(b->e);
  delete b;
  return CLF_OK;
}

}  // extern "C"
