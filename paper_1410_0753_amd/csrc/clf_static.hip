// No-allocation variant of clf_step (include/clf.h: clf_step_static).
//
// The step kernel needs device memory beyond the caller's state: the grid
// descriptor, the non-finite flag, the metric arrays (inverse spacings, row
// factors, tan(lat)/R) and the XCD-ordered tile list.  A context keeps them in
// the caller's workspace; here they live in one file-scope device array of
// fixed size, so the call allocates nothing.  Each GPU the library runs on
// holds its own copy of the array until the process ends; every call on that
// GPU shares it and leaves its contents behind, so calls that overlap on one
// GPU (on different streams or threads) race.
#include "clf.h"
#include "clf_internal.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

// Scratch of the no-allocation entry point: descriptor, flag, metrics, tiles.
constexpr size_t kStaticScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace clf {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
// Device address of `scratch` on each device (looked up once, with that
// device current), and a host copy of the descriptor, metrics and tiles that
// the device's scratch holds, so that a call repeating the last call's grid
// and buffers uploads nothing.
void* g_scratch_dev[kMaxDevices];
std::vector<unsigned char> g_scratch_image[kMaxDevices];

__global__ void clear_flag_kernel(StepState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->bad = 0;
}

int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_init_error(buf);
  return code;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

template <class R>
void put_array(std::vector<unsigned char>& img, size_t off, const std::vector<double>& v) {
  for (size_t i = 0; i < v.size(); ++i) {
    const R r = (R)v[i];
    std::memcpy(img.data() + off + i * sizeof(R), &r, sizeof(R));
  }
}

}  // namespace
}  // namespace clf

extern "C" int clf_step_static(const clf_grid* g, const clf_params* p, double dt,
                               const void* depth, void* h_a, void* u_a, void* v_a, void* h_b,
                               void* u_b, void* v_b, void* eta_max, void* speed2_max, int nsteps,
                               void* stream, int* nonfinite) {
  using namespace clf;
  int rc = validate_args(g, p);
  if (rc) return rc;
  if (!(dt > 0.0) || !(dt < 1e300)) return sfail(CLF_EINVAL, "dt must be > 0 and finite");
  if (nsteps < 0) return sfail(CLF_EINVAL, "negative step count");
  if (p->sweep_order != CLF_ORDER_XY)
    return sfail(CLF_EINVAL, "clf_step_static runs the x-y order only");
  if (!depth || !h_a || !u_a || !v_a || !h_b || !u_b || !v_b)
    return sfail(CLF_EINVAL, "null depth or state pointer");
  if ((eta_max == nullptr) != (speed2_max == nullptr))
    return sfail(CLF_EINVAL, "give both maxwave arrays or neither");
  const int fp32 = p->precision == CLF_FP32;
  const size_t es = fp32 ? 4 : 8;
  const int nx = g->nx, ny = g->ny;

  // scratch layout: descriptor, flag, six metric arrays, tiles
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t o_gd = take(sizeof(GridDesc)), o_st = take(sizeof(StepState));
  const size_t o_xib = take(es * (nx + 1)), o_xisb = take(es * nx), o_xfac = take(es * ny);
  const size_t o_yib = take(es * (ny + 1)), o_yisb = take(es * ny), o_tanR = take(es * ny);
  const size_t o_tiles = o;
  if (o_tiles >= kStaticScratchBytes)
    return sfail(CLF_ENOSPACE, "grid %dx%d: metric arrays exceed the %zu-byte static scratch", nx,
                 ny, kStaticScratchBytes);
  const size_t tile_room = (kStaticScratchBytes - o_tiles) / sizeof(Tile);

  const int flags = grid_flags(*g, *p);
  int seg = grid_default_segment(nx, ny, fp32, flags);
  int nblocks = 0;
  std::vector<Tile> tiles = grid_tiles(nx, ny, seg, &nblocks);
  while (tiles.size() > tile_room && seg < ny) {
    seg = seg * 2 < ny ? seg * 2 : ny;
    tiles = grid_tiles(nx, ny, seg, &nblocks);
  }
  if (tiles.size() > tile_room)
    return sfail(CLF_ENOSPACE, "grid %dx%d: tile list exceeds the %zu-byte static scratch", nx, ny,
                 kStaticScratchBytes);
  if (nsteps == 0) return CLF_OK;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sfail(CLF_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return sfail(CLF_EINVAL, "device index %d too large", dev);
  hipStream_t s = (hipStream_t)stream;

  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_scratch_dev[dev]) {
    // the array's name is a host-side stand-in: its device address on this
    // device is looked up once, with the device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return sfail(CLF_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  char* base = (char*)g_scratch_dev[dev];

  // host image of the scratch (the flag is cleared by a kernel each call)
  GridMetrics M;
  build_metrics(*g, *p, M);
  GridDesc gd{};
  gd.nx = nx;
  gd.ny = ny;
  gd.flags = flags;
  gd.maxout = 1;
  gd.H[0] = h_a; gd.H[1] = h_b;
  gd.U[0] = u_a; gd.U[1] = u_b;
  gd.V[0] = v_a; gd.V[1] = v_b;
  gd.D = const_cast<void*>(depth);
  gd.emax = eta_max;
  gd.smax2 = speed2_max;
  gd.xib = base + o_xib;
  gd.xisb = base + o_xisb;
  gd.xfac = base + o_xfac;
  gd.yib = base + o_yib;
  gd.yisb = base + o_yisb;
  gd.tanR = base + o_tanR;
  set_step_constants(gd, dt, *p);
  std::vector<unsigned char> img(o_tiles + tiles.size() * sizeof(Tile), 0);
  std::memcpy(img.data() + o_gd, &gd, sizeof gd);
  const std::pair<size_t, const std::vector<double>*> arrays[] = {
      {o_xib, &M.xib}, {o_xisb, &M.xisb}, {o_xfac, &M.xfac},
      {o_yib, &M.yib}, {o_yisb, &M.yisb}, {o_tanR, &M.tanR}};
  for (const auto& a : arrays) {
    if (fp32) put_array<float>(img, a.first, *a.second);
    else put_array<double>(img, a.first, *a.second);
  }
  std::memcpy(img.data() + o_tiles, tiles.data(), tiles.size() * sizeof(Tile));
  if (g_scratch_image[dev] != img) {
    // stream-ordered after earlier work on this stream; the wait lets the
    // host image go out of scope
    e = hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      g_scratch_image[dev].clear();
      return sfail(CLF_EHIP, "scratch upload: %s", hipGetErrorString(e));
    }
    g_scratch_image[dev].swap(img);
  }

  StepState* st = (StepState*)(base + o_st);
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(64), 0, s, st);
  e = hipGetLastError();
  const int order = step_order_for(nx, ny);
  const int do_max = eta_max != nullptr;
  for (int k = 0; k < nsteps && e == hipSuccess; ++k)
    e = launch_step(fp32, order, flags, (const GridDesc*)(base + o_gd),
                    (const Tile*)(base + o_tiles), (int)tiles.size(), st, k & 1, do_max, nblocks,
                    s);
  if (e != hipSuccess) return sfail(CLF_EHIP, "step launch: %s", hipGetErrorString(e));
  if (nonfinite) {
    StepState h{};
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&h, st, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return sfail(CLF_EHIP, "non-finite flag: %s", hipGetErrorString(e));
    *nonfinite = h.bad ? 1 : 0;
  }
  return CLF_OK;
}
