// Internal declarations shared by the host runtime and the HIP kernels of
// the split-step library.  Not part of the public ABI (include/clf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "clf.h"

namespace clf {

// node flags inside the sweeps
enum : int {
  F_EX = 1,    // node exists (inside the grid)
  F_WET = 2,   // wet
  F_FIX = 4,   // forcing ring node: held, not updated by the sweeps
  F_FLD = 8,   // flooded in step (b) of this sweep
  F_OPEN = 16, // outside the grid beyond an open (radiating) edge
};

// grid flags
enum : int {
  G_FIX_W = 1,
  G_FIX_E = 2,
  G_FIX_S = 4,
  G_FIX_N = 8,
  G_WALLMODE = 16,  // itopo = 0: nodes shallower than dwall never flood
  G_SOLVER1 = 32,
  G_SPHSRC = 64,    // tan(lat) continuity source in the y-sweep
  G_FRICTION = 128,
  G_WIDE = 256,     // field arrays above 4 GiB: 64-bit addresses in the step kernel
  G_TINYH = 512,    // FP64 with h_min below 1e-200: wet depths may need the
                    // small-argument path of the square root
  G_FRIC_SEMI = 1024,  // friction in the semi-implicit form (option) instead of -alpha dt
  G_OPEN_W = 2048,     // open (radiating) edges
  G_OPEN_E = 4096,
  G_OPEN_S = 8192,
  G_OPEN_N = 16384,
  G_OPEN_ANY = G_OPEN_W | G_OPEN_E | G_OPEN_S | G_OPEN_N,
  G_LDSROWS = 32768,   // FP32 2-D march: rows staged in LDS by direct global-to-LDS
                       // loads (a launch mode; the results are the same bits)
};

// kernel orders
enum : int { ORD_XY = 0, ORD_YX = 1, ORD_X = 2, ORD_Y = 3 };

// Per-grid descriptor, resident in device memory.  Field arrays are either
// double (FP64 contexts) or float (FP32 contexts).
struct GridDesc {
  int nx, ny;
  int flags;
  int maxout;
  void* H[2];   // FP64: water column height h; FP32: surface eta
  void* U[2];
  void* V[2];
  void* D;      // depth (+down)
  void* emax;   // running max of eta
  void* smax2;  // running max of u^2 + v^2
  const void* xib;   // [nx+1] 1/Delta x_{k-1}
  const void* xisb;  // [nx]   1/(Delta x_{k-1} + Delta x_k)
  const void* xfac;  // [ny]   row factor on the x inverse spacings
  const void* yib;   // [ny+1]
  const void* yisb;  // [ny]
  const void* tanR;  // [ny]   tan(lat)/R (zeros when the source is off)
  double dt, hdt, dt2, hmin, gn2, inv16g, dwall;
  // gauges whose records the step kernel writes: [ngauge][3] (row, column,
  // gauge index), grouped by tile (Tile::g0, gn); records [slot][ngauge][3]
  const int* gtab;
  double* grec;
  int ngauge;
  int pad_g;
};

// Per-context device flags.
struct StepState {
  int bad;           // a non-finite value was written
  int pad[3];
};

// Work tile of one wavefront: grid index, first output column, first
// output row, number of output rows; the tile's gauges are entries
// [g0, g0 + gn) of its grid's gauge table.
struct Tile {
  int grid, x0, y0, rows;   // grid | kTileReverse: the segment marches rows downward
  int g0, gn, pad0, pad1;
};
constexpr int kTileReverse = 1 << 30;

// Per-point sampling tables.
struct SampleDesc {
  int ngauge;
  int gout;
  int npts;          // enclosed-grid boundary points (all grids, all sides)
  int bndout;
  const long long* gidx;  // [ngauge] node index iy*nx + ix
  double* grec;      // [cap][ngauge][3]
  int gcap;
  const long long* sidx;  // [npts][4] corner node indices
  const double* swt;      // [npts][4] corner weights
  const int* sout;        // [npts] offset of the point inside a record: q*np + k within its side block
  double* srec;           // [cap][rec_len]
  int rec_len;
  int scap;
  int grid;               // grid index in the descriptor table
  long long g_first;      // first gauge record level
  long long s_first;      // first enclosed-grid record level
};

// Forcing tables (per side).
struct ForceDesc {
  int nt[4];
  int np[4];
  const double* t[4];
  const double* vals[4];  // [nt][3][np]
  int grid;
};

constexpr int WAVE = 64;
constexpr int HALO = 3;
constexpr int STRIP = WAVE - 2 * HALO;  // output columns per wavefront
constexpr int WAVES_PER_BLOCK = 4;

// Kernel launchers (clf_kernels.hip).
// rec_slot >= 0: the step writes the gauge records of that slot (the level
// the step reaches); -1: no records.
hipError_t launch_step(int fp32, int order, int gflags, const GridDesc* grids, const Tile* tiles,
                       int ntiles, StepState* st, int parity, int do_max, int nblocks,
                       hipStream_t s, int rec_slot = -1);
// Resident workgroups per compute unit of the step kernel variant.
hipError_t step_blocks_per_cu(int fp32, int order, int gflags, int* n);
hipError_t launch_init_state(int fp32, const GridDesc* gd_host, const GridDesc* gd_dev,
                             const double* eta, const double* u, const double* v, int deform,
                             long long N, int parity, hipStream_t s);
hipError_t launch_set_raw(int fp32, const GridDesc* gd_host, const GridDesc* gd_dev,
                          const double* h, const double* u, const double* v, long long N,
                          int parity, hipStream_t s);
hipError_t launch_get_raw(int fp32, const GridDesc* gd_host, const GridDesc* gd_dev, double* h,
                          double* u, double* v, long long N, int parity, hipStream_t s);
hipError_t launch_get_state(int fp32, const GridDesc* gd_host, const GridDesc* gd_dev,
                            double* eta, double* u, double* v, uint8_t* wet, long long N,
                            int parity, hipStream_t s);
hipError_t launch_read_maxwave(int fp32, const GridDesc* gd_host, const GridDesc* gd_dev,
                               double* emax, double* smax, long long N, hipStream_t s);
hipError_t launch_get_depth(int fp32, const GridDesc* gd_host, const GridDesc* gd_dev, double* d,
                            long long N, hipStream_t s);
hipError_t launch_clear_maxwave(int fp32, const GridDesc* gd_host, long long N, hipStream_t s);
// Records of level n: the gauges (when do_gauges) and the enclosed-grid series.
hipError_t launch_sample(int fp32, const GridDesc* gd_dev, const SampleDesc* sd_dev, int nthreads,
                         long long n, int parity, int do_gauges, hipStream_t s);
hipError_t launch_forcing(int fp32, const GridDesc* gd_dev, const ForceDesc* fd_dev, int nthreads,
                          long long n, int parity, hipStream_t s);
hipError_t launch_deform_depth(int fp32, const GridDesc* gd_host, const double* eta, long long N,
                               hipStream_t s);

// One halo copy of a y-band decomposition: HALO rows of (h, u, v) from row
// src_row of member src to row dst_row of member dst (rows of the members'
// own grids).
struct BandXchg {
  int src, src_row, dst, dst_row;
};
hipError_t launch_band_exchange(int fp32, const GridDesc* grids, const BandXchg* xt, int nxchg,
                                int nx, int parity, hipStream_t s);

// Host helpers of the runtime (clf_runtime.cpp), shared with the
// no-allocation entry point (clf_static.hip).
struct GridMetrics {
  // inverse spacings: x [nx+1], [nx]; row factor [ny]; y [ny+1], [ny]; tan(lat)/R [ny]
  std::vector<double> xib, xisb, xfac, yib, yisb, tanR;
};
void build_metrics(const clf_grid& g, const clf_params& p, GridMetrics& m);
int grid_flags(const clf_grid& g, const clf_params& p);
void set_step_constants(GridDesc& gd, double dt, const clf_params& p);
// XCD-ordered tile list of one grid for a segment length; *nblocks receives
// the workgroup count of a launch that covers it
std::vector<Tile> grid_tiles(int nx, int ny, int seg, int* nblocks);
int grid_default_segment(int nx, int ny, int fp32, int gflags);
int step_order_for(int nx, int ny);
int validate_args(const clf_grid* g, const clf_params* p);
void set_init_error(const char* msg);

// Flags used by the adjoint sweep (bytes; zero them once before the first
// sweep, every sweep leaves them zero).
int adjoint_flag_count(int nx, int ny);
hipError_t launch_adjoint_sweep(const GridDesc* gd_host, int axis, const double* preH,
                                const double* preU, const double* preV, const double* lamH,
                                const double* lamU, const double* lamV, double* outH,
                                double* outU, double* outV, unsigned char* flags, hipStream_t s);
hipError_t launch_inject(const GridDesc* gd_host, const double* H, const long long* gidx, int ng,
                         const double* rec_adj, double* lamH, double* lamU, double* lamV,
                         hipStream_t s);
hipError_t launch_initial_adjoint(const GridDesc* gd_host, const double* H0, const double* lamH,
                                  const double* lamU, const double* lamV, double* dEta, double* dU,
                                  double* dV, long long N, hipStream_t s);

}  // namespace clf
