/*
 * clf.h -- C-ABI of the MI355X split-step shallow-water library.
 *
 * The library advances the nonlinear shallow-water equations (paper section
 * Numerics, eq1/eqABC: W_t = A W_x + B W_y + C with W = (h, u, v)) by the
 * dimensionally split VTCS-2 scheme: per time step a 1-D sweep along x on
 * every row (eq2A) then a 1-D sweep along y on every column (eq2B), each
 * sweep advancing the Riemann invariants p = u + 2 sqrt(gh), q = u - 2 sqrt(gh)
 * and the tangential velocity (pq1-pq3) with the depth-balanced difference
 * Q (eqQ) and the solver2 stencil (or solver1), recovering u = (p+q)/2 and
 * h = (p-q)^2/16g (stateu, stateh), inside the moving-cliff wet/dry cycle
 * (a)-(e) of section Inundation algorithm.  Bathymetry is preprocessed at
 * init against the depth-jump instability (section Numerical stability:
 * dstab, newdw, newdc).  Outputs follow the paper's Running Options:
 * maxwave, virtual gauges, boundary series for enclosed grids.
 *
 * Conventions
 *   - Grids are row-major [ny][nx], x (longitude) fastest; depth is positive
 *     down, negative on land (Running Options, Bathymetry data).
 *   - Units: metres, seconds, decimal degrees for lon/lat.
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are host memory, read or written during the call.
 *   - The caller owns every buffer.  The library places all its device data
 *     in the caller's workspace (size from clf_workspace_bytes) and
 *     allocates no device memory itself.
 *   - All device work is enqueued on the stream given at init (a
 *     hipStream_t passed as void*).  clf_step returns asynchronously;
 *     device-detected errors (non-finite state) surface at the next
 *     clf_sync, clf_get_state, clf_read_* or clf_get_raw_state.
 *   - Every call returns CLF_OK (0) or a negative error code;
 *     clf_last_error gives a message.  No exception crosses the ABI.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CLF_H
#define CLF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define CLF_OK 0
#define CLF_EINVAL (-1)      /* bad shape, argument or coordinate */
#define CLF_ECFL (-2)        /* still-water Courant number above the limit */
#define CLF_EHIP (-3)        /* a HIP runtime call failed */
#define CLF_ENONFINITE (-4)  /* the state became non-finite on the device */
#define CLF_ESTATE (-5)      /* call made in the wrong order */
#define CLF_ENOSPACE (-6)    /* workspace or record capacity too small */
#define CLF_ESSL (-7)        /* depth preprocessing did not converge */

/* coordinate systems (parameter file item 1) */
#define CLF_CARTESIAN 0
#define CLF_SPHERICAL 1

/* arithmetic of the state and of the sweeps */
#define CLF_FP64 0
#define CLF_FP32 1

/* split order: x then y every step, or x-y / y-x on even / odd steps */
#define CLF_ORDER_XY 0
#define CLF_ORDER_ALTERNATE 1

/* sides of a grid */
#define CLF_WEST 0
#define CLF_EAST 1
#define CLF_SOUTH 2
#define CLF_NORTH 3

/* clf_query keys */
#define CLF_Q_MAX_CFL 1        /* max still-water Courant number sqrt(g d) dt / dx */
#define CLF_Q_SSL_PASSES 2     /* passes of the depth preprocessing (0 if off) */
#define CLF_Q_STEP 3           /* time steps done since clf_set_initial */
#define CLF_Q_MIN_F 4          /* min over wet interior nodes of f_j (eq:f), both axes */
#define CLF_Q_WORKSPACE 5      /* workspace bytes in use */
#define CLF_Q_GAUGE_RECORDS 6  /* gauge records held */
#define CLF_Q_TILES 7          /* wavefront tiles per step kernel launch */
#define CLF_Q_SEGMENT 8        /* rows per wavefront tile (autotuned) */
#define CLF_Q_BLOCKS 9         /* workgroups per step kernel launch */
#define CLF_Q_GRAPH_REPLAYS 10 /* hipGraph replays issued so far */
#define CLF_Q_WIDE 11          /* 1 if the step kernel runs its 64-bit-address variant */
/* With kernel_timing = 1: mean duration (ms) of the step-kernel launches of
 * clf_step since the last reset, from a HIP event pair recorded around each
 * launch on the context's stream (waits for them); their count; and a reset
 * (returns the count before it). */
#define CLF_Q_KERNEL_MS 12
#define CLF_Q_KERNEL_LAUNCHES 13
#define CLF_Q_KERNEL_RESET 14
/* 1 if the FP32 step kernel stages the rows of its march in LDS (FP32 grids
 * whose fields exceed the 256 MiB last-level cache; the environment variable
 * CLF_LDS_ROWS=0 or 1, read at init, forces it off or on).  The results are
 * the same bits either way. */
#define CLF_Q_LDS_ROWS 15

typedef struct clf_ctx clf_ctx;

/* Grid (Running Options: Bathymetry data; parameter file item 1).
 * x[nx], y[ny] are host arrays, strictly increasing: metres (Cartesian) or
 * decimal degrees (spherical lon/lat).  A 2-D grid needs nx, ny >= 3; a 1-D
 * grid has nx == 1 or ny == 1 and at least 3 nodes along the other axis.
 * nx * ny must be below 2^32; larger grids are rejected with CLF_EINVAL.
 * Grids whose field arrays exceed 4 GiB (nx * ny * 8 in FP64, * 4 in FP32)
 * run a variant of the step kernel with 64-bit addresses, which carries every
 * option and is somewhat slower (CLF_Q_WIDE reports it).  The environment
 * variable CLF_WIDE_OFFSETS=1, read at init, selects that variant for any
 * grid. */
typedef struct clf_grid {
  int32_t nx, ny;
  int32_t coord;
  const double* x;
  const double* y;
} clf_grid;

/* Parameters (parameter file items 5-18 and the depth_ssl options).
 * clf_default_params fills every field; change what you need. */
typedef struct clf_params {
  int32_t precision;        /* CLF_FP64 or CLF_FP32 */
  double h_min;             /* item ground: flow depth at or below which a node is dry (> 0);
                               FP64 grids with h_min below 1e-200 run the general (slower)
                               step kernel, whose square root handles arguments under 2^-767 */
  double manning_n2;        /* item crough: Manning n^2; 0 disables friction */
  int32_t itopo;            /* item itopo: 1 inundation; 0 vertical wall at depth dwall */
  double dwall;             /* item dwall: nodes shallower than this are land when itopo = 0 */
  double ssl_alpha;         /* preprocessing limit alpha (dstab); 0 disables it; default 2 */
  double ssl_min_depth;     /* preprocessing minimal wet depth, default 0.1 m */
  int32_t sweep_order;      /* CLF_ORDER_XY (default) or CLF_ORDER_ALTERNATE */
  int32_t solver;           /* 2 = solver2 (default, current Cliffs), 1 = solver1 */
  double earth_radius;      /* metres, default 6371000 */
  int32_t spherical_metric; /* 1: tan(lat) continuity source in the y-sweep (default) */
  double cfl_limit;         /* clf_init fails with CLF_ECFL above this, default 1 */
  int32_t maxout;           /* item maxout: steps between maxwave updates (>= 1) */
  int32_t gout;             /* item gout: steps between gauge records (>= 1) */
  int32_t bndout;           /* item bndout: steps between enclosed-grid records (>= 1) */
  int32_t max_gauges;       /* capacity: gauges */
  int32_t gauge_capacity;   /* capacity: gauge records held before clf_clear_records */
  int32_t max_enclosed;     /* capacity: enclosed grids */
  int32_t max_enclosed_points; /* capacity: boundary points summed over enclosed grids */
  int32_t series_capacity;  /* capacity: enclosed-grid records held */
  int32_t forcing_capacity; /* capacity: time levels per forcing side (0: no forcing) */
  int32_t segment;          /* rows per wavefront tile of the step kernel, 8..4096; 0 =
                               automatic: the shortest segment whose tiles fit one wave of
                               resident workgroups on this GPU */
  int32_t autotune;         /* 1: clf_init times candidate tile shapes on this grid and keeps
                               the fastest (cached per grid size and precision in the process) */
  int32_t graph_steps;      /* >0: step sequences that do not depend on the step index (no
                               forcing, no gauges or series, maxout 1, x-y order) run as
                               replays of a hipGraph holding this many steps (even); 0: off */
  int32_t persistent_blocks; /* >0: the step kernel runs this many workgroups (a multiple of 8)
                               looping over the tiles; 0: one wavefront per tile */
  int32_t friction_form;    /* bottom friction (manning_n2 > 0): 0 (default) the -alpha_j dt term
                               of solver2 / solver1 on p and q, alpha = g n^2 w |U| / h^(4/3) at the
                               old time level; 1 semi-implicit option w' / (1 + dt alpha / w),
                               unconditionally damping in thin layers */
  int32_t open_sides;       /* open (radiating) edges, not in the paper: bit mask 1 W, 2 E, 4 S,
                               8 N.  The ghost beyond an open edge carries the edge node's
                               outgoing Riemann invariant and the still-water incoming one
                               (p0 = 2 sqrt(g d) from the west/south, q0 = -2 sqrt(g d) from the
                               east/north).  Other edges are walls.  Grids with open edges run the
                               general (slower) step kernel; the adjoint rejects them. */
  int32_t kernel_timing;    /* 1: clf_step records a HIP event pair around each step-kernel
                               launch (CLF_Q_KERNEL_MS); step sequences then run without
                               hipGraphs.  Default 0. */
} clf_params;

void clf_default_params(clf_params* p);

/* Row-major index iy * nx + ix of node (ix, iy), 0-based, computed in 64 bits
 * (grids hold up to 2^32 - 1 nodes).  CLF_EINVAL if the node is outside an
 * nx x ny grid or index is NULL.  Host only; the library indexes gauges this
 * way. */
int clf_node_index(int nx, int ny, int ix, int iy, int64_t* index);

/* Device workspace needed by clf_init for this grid and these parameters. */
int clf_workspace_bytes(const clf_grid* g, const clf_params* p, size_t* bytes);

/* Create a context.  depth: host [ny][nx] (+down, negative = land).  dt: time
 * step (item dt).  The depth is preprocessed (dstab/newdw/newdc) when
 * p->ssl_alpha > 0, metric arrays are built, and the still-water Courant
 * number |lambda| dt / dx (stability remark after solver2) is checked
 * against p->cfl_limit (CLF_ECFL).  stream: hipStream_t (NULL = default
 * stream).  ws: device workspace of ws_bytes >= clf_workspace_bytes, owned
 * by the caller and kept alive until clf_destroy.  The state starts as the
 * lake at rest. */
int clf_init(clf_ctx** out, const clf_grid* g, const double* depth, double dt,
             const clf_params* p, void* stream, void* ws, size_t ws_bytes);

/* Initial conditions (Running Options: input to the computations; item
 * quake).  eta, u, v: device [ny][nx] FP64 arrays or NULL for zero.  With
 * deform_bottom = 0 the deformation eta is applied to the free surface
 * (h = max(d + eta, 0)); with 1 to the sea floor (d <- d - eta, h = max(d, 0)).
 * Nodes with h <= h_min are dry.  Resets the step counter, maxwave and
 * records. */
int clf_set_initial(clf_ctx* c, const double* eta, const double* u, const double* v,
                    int deform_bottom);

/* Restart: raw state h (water column height), u, v as device [ny][nx] FP64
 * arrays, and the step index n it belongs to.  clf_get_raw_state then
 * clf_set_raw_state continues a run bit for bit (FP64). */
int clf_set_raw_state(clf_ctx* c, const double* h, const double* u, const double* v, int64_t n);
int clf_get_raw_state(clf_ctx* c, double* h, double* u, double* v);

/* Boundary forcing (Running Options: boundary time-series, layout
 * vals(tim,uvq,pnt)).  side: CLF_WEST/EAST (np = ny) or CLF_SOUTH/NORTH
 * (np = nx).  t[nt] strictly increasing model times (host), vals host
 * [nt][3][np] with uvq = (u, v, eta).  At the start of every step the outer
 * ring node of that side takes the values interpolated linearly in time at
 * t = n dt (held constant outside the series) and is not updated by the
 * sweeps.  Requires p->forcing_capacity >= nt. */
int clf_set_boundary_forcing(clf_ctx* c, int side, int nt, const double* t, const double* vals);

/* Virtual gauges (items Ngages, gout, and the index list; 0-based here).
 * ix, iy: host int32 [n].  A record (eta, u, v) of every gauge is taken at
 * each step index n with n % gout == 0 (including n = 0); dry nodes record
 * zeros. */
int clf_set_gauges(clf_ctx* c, int n, const int32_t* ix, const int32_t* iy);

/* Enclosed grid (items nests and the grid names; output boundary series
 * files).  x[nx], y[ny]: host coordinates inside the master grid.  Every
 * bndout steps the library records (u, v, eta) along the four sides (W and
 * E along y, S and N along x) by bilinear interpolation over the wet
 * corners of the enclosing master cell (all dry: zeros).  *id receives the
 * grid's index. */
int clf_add_enclosed_grid(clf_ctx* c, int nx, int ny, const double* x, const double* y, int* id);

/* Advance nsteps split steps (items dt, steps_total).  Asynchronous. */
int clf_step(clf_ctx* c, int nsteps);

/* One sweep only (axis 0: x-sweep of every row, eq2A; 1: y-sweep of every
 * column, eq2B), without forcing, sampling or step counting.  Diagnostics. */
int clf_sweep(clf_ctx* c, int axis);

/* State at the current step: eta = h - d on wet nodes, 0 on dry ones; u, v
 * (0 on dry nodes); wet = 1 where h > h_min.  Device arrays [ny][nx]; any
 * may be NULL.  Synchronises the stream. */
int clf_get_state(clf_ctx* c, double* eta, double* u, double* v, uint8_t* wet);

/* Depth in use (after preprocessing and any sea-floor deformation), device. */
int clf_get_depth(clf_ctx* c, double* d);

/* Gauge records (output gauges file): host out [nrec][ng][3] (eta, u, v),
 * times [nrec] = n dt; *nrec receives the count (at most max_rec copied). */
int clf_read_gauges(clf_ctx* c, double* out, double* times, int* nrec, int max_rec);

/* Maxwave (output maxwave file): running maxima over wet nodes of eta and of
 * the current speed sqrt(u^2 + v^2), updated after every step n with
 * n % maxout == 0; both start at 0.  Device [ny][nx] FP64; either may be NULL. */
int clf_read_maxwave(clf_ctx* c, double* eta_max, double* speed_max);

/* Enclosed-grid series of one side: host vals [nrec][3][np], times [nrec]. */
int clf_read_boundary_series(clf_ctx* c, int id, int side, double* vals, double* times,
                             int* nrec, int max_rec);

/* Drop held gauge and enclosed-grid records (capacity is reused). */
int clf_clear_records(clf_ctx* c);

/* Wait for the stream; report CLF_ENONFINITE if the state went non-finite. */
int clf_sync(clf_ctx* c);

/* Scalar diagnostics (CLF_Q_*). */
int clf_query(clf_ctx* c, int what, double* value);

/* Message of the last error on this context (or of the last failed
 * clf_init when c is NULL).  Valid until the next call on c. */
const char* clf_last_error(const clf_ctx* c);

/* Free host-side resources.  The workspace stays the caller's. */
int clf_destroy(clf_ctx* c);

/* ------------------------------------------------------------------------
 * No-allocation variant of clf_step, for callers that cannot allocate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It runs the same split step (same kernels, same results bit for
 * bit as clf_step on a context with the same grid, depth and parameters) on
 * state arrays the caller owns, and needs no context and no workspace: the
 * grid descriptor, the non-finite flag, the metric arrays and the tile list
 * go into a fixed static scratch array of 4 MiB on each GPU (held until the
 * process ends).  The call allocates no device memory and calls no
 * allocating routine.
 *
 *   g, p, dt   grid, parameters and time step as for clf_init.  Not done
 *              here: depth preprocessing (pass a preprocessed depth, e.g. from
 *              clf_get_depth of a context), the Courant check, forcing,
 *              gauges, enclosed grids; p->sweep_order must be CLF_ORDER_XY.
 *   depth      device [ny][nx] in the storage precision (double for CLF_FP64,
 *              float for CLF_FP32), +down, used as given.
 *   h_a,u_a,v_a, h_b,u_b,v_b
 *              two device state buffers [ny][nx] in the storage form: FP64
 *              h, u, v as double; FP32 eta = h - d (dry nodes hold -d), u, v
 *              as float.  Buffer A holds the state on entry; the steps
 *              alternate A -> B -> A ..., so on return the state is in A if
 *              nsteps is even and in B if it is odd.  Buffers must not overlap.
 *   eta_max, speed2_max
 *              device [ny][nx] running maxima (storage precision) of eta and
 *              of u^2 + v^2 over wet nodes, updated after every step; both
 *              NULL to skip.  The caller initialises them (zeros).
 *   nsteps     steps to take (>= 0).
 *   stream     hipStream_t (as void*) on the current device; the call is
 *              asynchronous unless nonfinite is given.
 *   nonfinite  NULL, or a host int that receives 1 if the state went
 *              non-finite during the call (the call then waits for the stream).
 *
 * Returns CLF_EINVAL for bad arguments, CLF_ENOSPACE when the grid's metric
 * arrays and tile list do not fit the 4 MiB scratch (about nx + ny above
 * 100000 in FP64), CLF_EHIP on a runtime error; clf_last_error(NULL) gives
 * the message.  All calls on one GPU share its scratch, which keeps the last
 * call's contents (a call that repeats the previous call's grid and buffers
 * uploads nothing): calls that overlap on one GPU, on different streams or
 * threads, race. */
int clf_step_static(const clf_grid* g, const clf_params* p, double dt, const void* depth,
                    void* h_a, void* u_a, void* v_a, void* h_b, void* u_b, void* v_b,
                    void* eta_max, void* speed2_max, int nsteps, void* stream, int* nonfinite);

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of the FP64 split step, for gradients of a loss of
 * the gauge records with respect to the initial state (source inversion).
 * The branch decisions of the wet/dry cycle and of stateh are frozen at the
 * forward values; the forward run keeps a checkpoint of the state every
 * ckpt_every steps (default ceil(sqrt(nsteps))) and the reverse run
 * recomputes each segment from its checkpoint.  Requires an FP64 context,
 * the x-y order and no boundary forcing; the initial condition must be a
 * free-surface deformation (deform_bottom = 0).
 * ------------------------------------------------------------------------ */

/* Device workspace for an adjoint run of nsteps (caller-owned). */
int clf_adjoint_workspace_bytes(const clf_ctx* c, int nsteps, int ckpt_every, size_t* bytes);

/* Forward run of nsteps from the state set by clf_set_initial (step 0),
 * recording gauges as clf_step does and storing checkpoints in ws. */
int clf_adjoint_forward(clf_ctx* c, int nsteps, int ckpt_every, void* ws, size_t ws_bytes);

/* Reverse run.  rec_adj: host [nrec][ng][3], the derivative of the loss with
 * respect to every gauge record (eta, u, v) of the forward run (nrec must be
 * the number of records it took).  Outputs: device [ny][nx] FP64 gradients
 * with respect to the initial surface deformation eta0 and the initial
 * velocities u0, v0 (any may be NULL).  Synchronises the stream. */
int clf_adjoint_backward(clf_ctx* c, const double* rec_adj, int nrec, double* d_eta0,
                         double* d_u0, double* d_v0);

/* ------------------------------------------------------------------------
 * Ensemble: many independent grids (scenarios) of uneven sizes advanced in
 * lockstep.  Each time step is ONE launch of the step kernel over the
 * concatenated tile list of all members (XCD-aware order, optionally a
 * persistent grid-stride launch), and step chunks are replayed from a
 * hipGraph when p->graph_steps > 0 and maxout == 1.  Every member computes
 * exactly what a single-grid context would (bit for bit).  Members have
 * their own grid, depth and dt and share the parameters; gauges, series
 * and forcing are not available on ensemble members (maxwave is).
 * ------------------------------------------------------------------------ */
typedef struct clf_ens clf_ens;

/* Workspace for n members (grids[i] as for clf_init). */
int clf_ensemble_workspace_bytes(int n, const clf_grid* grids, const clf_params* p,
                                 size_t* bytes);

/* depths[i]: host [ny_i][nx_i]; dts[i]: member time step.  Each member is
 * preprocessed and checked as by clf_init and starts as the lake at rest. */
int clf_ensemble_init(clf_ens** out, int n, const clf_grid* grids, const double* const* depths,
                      const double* dts, const clf_params* p, void* stream, void* ws,
                      size_t ws_bytes);

/* Initial condition of one member (as clf_set_initial); resets its maxwave. */
int clf_ensemble_set_initial(clf_ens* e, int member, const double* eta, const double* u,
                             const double* v, int deform_bottom);

/* Advance every member nsteps steps.  Asynchronous. */
int clf_ensemble_step(clf_ens* e, int nsteps);

/* Per-member read-outs (device arrays of that member's shape). */
int clf_ensemble_get_state(clf_ens* e, int member, double* eta, double* u, double* v,
                           uint8_t* wet);
int clf_ensemble_read_maxwave(clf_ens* e, int member, double* eta_max, double* speed_max);

int clf_ensemble_sync(clf_ens* e);
int clf_ensemble_query(clf_ens* e, int what, double* value);
const char* clf_ensemble_last_error(const clf_ens* e);
int clf_ensemble_destroy(clf_ens* e);

/* ------------------------------------------------------------------------
 * One grid split into y-bands (row ranges) on one device: the per-GPU part
 * of sharding a large grid over GPUs (the paper's splitting into independent
 * row and column problems, section Numerics, eq2A/eq2B).  The x-sweep is
 * row-local, and the y-sweep of a row needs the post-x state of HALO = 3
 * rows on each side (steps (a)-(e) reach 3 nodes), so each band holds its
 * own rows plus 3 halo rows beyond each inner edge.  A step is one launch of
 * the step kernel over all bands' tiles, then one exchange: the 3 rows of
 * (h, u, v) beyond each inner edge take the post-step values of the band
 * that owns them (on several GPUs this is the point-to-point exchange with
 * each neighbour).  Results are bit for bit those of a clf_init context on
 * the whole grid.  Depth preprocessing and the Courant check run once, on
 * the whole grid.  Bands use the x-y order; gauges, enclosed grids and
 * forcing are not available on them (maxwave is).  Every band needs at
 * least 3 rows.
 * ------------------------------------------------------------------------ */
typedef struct clf_bands clf_bands;

/* Workspace for grid g split into nbands bands (caller-owned, device). */
int clf_bands_workspace_bytes(const clf_grid* g, const clf_params* p, int nbands, size_t* bytes);

/* As clf_init, for the whole grid (depth: host [ny][nx]); rows are dealt to
 * the bands as evenly as possible, lower rows first. */
int clf_bands_init(clf_bands** out, const clf_grid* g, const double* depth, double dt,
                   const clf_params* p, int nbands, void* stream, void* ws, size_t ws_bytes);

/* As clf_set_initial, with whole-grid device arrays [ny][nx]. */
int clf_bands_set_initial(clf_bands* b, const double* eta, const double* u, const double* v,
                          int deform_bottom);

/* Advance nsteps steps (step launch + halo exchange each).  Asynchronous. */
int clf_bands_step(clf_bands* b, int nsteps);

/* As clf_get_state and clf_read_maxwave, into whole-grid device arrays
 * (each band writes its own rows).  Synchronise the stream. */
int clf_bands_get_state(clf_bands* b, double* eta, double* u, double* v, uint8_t* wet);
int clf_bands_read_maxwave(clf_bands* b, double* eta_max, double* speed_max);

int clf_bands_sync(clf_bands* b);
/* CLF_Q_MAX_CFL, CLF_Q_MIN_F, CLF_Q_SSL_PASSES of the whole grid; CLF_Q_STEP,
 * CLF_Q_TILES, CLF_Q_SEGMENT, CLF_Q_BLOCKS, CLF_Q_WIDE, CLF_Q_LDS_ROWS,
 * CLF_Q_WORKSPACE of the launch over all bands. */
int clf_bands_query(clf_bands* b, int what, double* value);
const char* clf_bands_last_error(const clf_bands* b);
int clf_bands_destroy(clf_bands* b);

#ifdef __cplusplus
}
#endif

#endif /* CLF_H */
