// gdg_internal.h -- data layout shared by the host setup and the HIP kernels
// of libgdg.  Not part of the public interface (include/gdg.h is).
//
// Stencil layout on the device: row-blocked ELL.  A block is R = C * nloc
// consecutive rows (C whole cells), the rows of one workgroup, so a cell's
// dofs are always in one workgroup (its consistent-mass block can be solved
// in LDS).  Every block has the same width W = nloc + dim * (k+1)^(dim-1), the
// widest row (a cell corner with all neighbours); narrower rows are padded.
// Slot t of row lane r in block b lives at index (b * W + t) * R + r, so the
// lanes of a wavefront read consecutive addresses for every slot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "gdg.h"

namespace gdg {

// slot kinds (low 3 bits of the meta byte)
enum : uint8_t {
  SK_PAD = 0,
  SK_CELL = 1,        // j in the same cell (the diagonal included); aux = local index of j
  SK_FACE_COLLOC = 2, // j across a face, x_j = x_i (topologically)
  SK_FACE = 3,        // j across a face, other node of that face
  SK_GHOST = 4        // boundary part: col = i, c = c_i^{d,k}; aux = its boundary class
};
static inline int meta_kind(uint8_t m) { return m & 7; }
static inline int meta_aux(uint8_t m) { return m >> 3; }
// Boundary class of a boundary part (the aux bits of its slot, 0 .. 29): the
// box face f whose data it takes and its kind (a gdg_bc other than PERIODIC).
__host__ __device__ inline int bclass(int f, int kind) { return (kind - 1) * 6 + f; }
__host__ __device__ inline int bclass_face(int c) { return c % 6; }
__host__ __device__ inline int bclass_kind(int c) { return c / 6 + 1; }

// One wavefront per workgroup: whole cells per block (the cell solve stays in
// LDS), and a finished wave's slot is refilled at once, which matters where
// the line searches of shock regions make the work per row uneven.
#ifndef GDG_BLOCK
#define GDG_BLOCK 64
#endif
constexpr int kBlockThreads = GDG_BLOCK;
constexpr int kMaxD = 3;
constexpr int kMaxNloc = 27;
constexpr int kMaxStages = 5;  // stages of a step (SSP-RK3: 3, SSPRK(5,4): 5)

// Control block in device memory.  In a device-driven run (captured graphs
// of several steps) the time loop state lives here too.
struct Ctl {
  unsigned long long taumin_bits[kMaxStages]; // per stage: min_i m_i / (2 |d_ii|) as IEEE bits
  double tau;                        // tau of the current step
  double dt_cap;                     // cap on tau (<= 0: none)
  double tau_fixed;                  // > 0: replaces the CFL rule in stage 1
  double t;                          // simulated time
  double t_final;                    // device-driven runs: end time
  long long steps;                   // steps completed
  long long step_limit;              // device-driven runs: stop after this many steps
  // Set when stage 2 or 3 finds tau above its CFL bound.  Every block of the
  // detecting kernel reaches the same decision from the same data, and later
  // kernels read it only at their start, so exits stay uniform.
  int cfl_flag;
  int bad_flag;                      // a state left A; read by the host only
  int viol_stage;
  int halt;                          // set by the step's first kernel: skip this step
  // Counters since the last upload: stage outputs of the limited scheme
  // outside their relaxed bounds (eq. local_bounds), pairs that limiter pass 1
  // cut (l_ij < 1), rows of quiet cells (every flux of the row exactly zero).
  // The kernels add into kCntSlots spread copies (KArgs::cnt); the statistics
  // call sums them here.
  unsigned long long bound_violations;
  unsigned long long limited_pairs;
  unsigned long long quiet_rows;
};
// Spread counters: counter c of slot s at cnt[(c * kCntSlots + s) * kCntStride]
// (one 128-byte line each).  A wavefront adds into the slot of its hardware
// block index, so that the device-scope atomics of the 8 XCDs meet at many
// addresses instead of one (integer sums: the totals do not depend on the
// order of the blocks).
constexpr int kCntSlots = 256, kCntStride = 16;
enum { kCntViolations = 0, kCntLimited = 1, kCntQuiet = 2, kCntKinds = 3 };
// Reduction of a state for the statistics call: per block partials, then one
// block combines them in a fixed order.  min rho, min eps, sum_i m_i U_i.
// Most cell rows in y of a 3D tile of the sweep order.
constexpr int64_t kTileRows = 64;
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;
constexpr int kRedFields = 2 + kMaxD + 2;
// Per-dof records (arrays of structures): the fields that a row gathers from
// its neighbours sit together, so that a neighbour costs one or two cache
// lines and a few wide loads instead of one line per field.
//  node record (kNodeStride doubles), two buffers: the stage input's and the
//  stage output's, chosen by the parity of nst * steps + stage (node_buffer):
//    [0, M) U, [M, M+D) velocity, then p, a, p^-alpha, f(s), s~, 1/p
//  bound record (kQStride): rho_min, rho_max, s~_min of the ring-1 partials, N_i
//  limiter record (kLimStride): [0, M) dU^H, [M, 2M) U^L, then rho_min,
//    rho_max, s~_min of the relaxed bounds, 1/(kappa_i m_i), N_i, and the
//    stage input U_i (everything a limiter pass needs of a row, in one place)
//  U^(1) record (kU1Stride): [0, M) the state after limiter pass 1
constexpr int kNodeStride = 16, kQStride = 4, kLimStride = 20, kU1Stride = 8;
template <int D> struct Rec {
  static constexpr int M = D + 2;
  // node record
  static constexpr int U = 0, u = M, p = 2 * D + 2, a = 2 * D + 3, pal = 2 * D + 4, fs = 2 * D + 5,
                       st = 2 * D + 6, ip = 2 * D + 7, nwide = D + 4;  // nwide: 16-byte loads of the whole record
  // limiter record
  static constexpr int dUH = 0, UL = M, B = 2 * M, ks = 2 * M + 3, N = 2 * M + 4, LU = 2 * M + 5,
                       nlim = 3 * M + 5;  // nlim: the limiter record's used doubles
  static_assert(ip < kNodeStride && nlim <= kLimStride && M <= kU1Stride, "record strides");
};

// Reference tables of one cell class (every cell of a uniform mesh).
struct RefTables {
  double mlump[kMaxNloc];                   // m_a
  double mblk[kMaxNloc * kMaxNloc];         // m_ab
  double minv[kMaxNloc * kMaxNloc];         // (M_K^{-1})_ab
  double cin[kMaxNloc * kMaxNloc * kMaxD];  // in-cell c_ab (a row, b column, axis)
  // across face f (0..5): for row a on face f and t-th node b of the touching
  // face of the neighbour: c vector, local index of b, collocation flag
  double cface[6 * kMaxNloc * 9 * kMaxD];
  int32_t bface[6 * 9];
  int32_t colloc[6 * kMaxNloc * 9];
  double cghost[6 * kMaxNloc * kMaxD];      // c_a^{d,f}
  int32_t onface[6 * kMaxNloc];             // 1 if node a lies on face f
  // per node a, from the scheme constants
  double hpk[kMaxNloc];    // c_k * hhat_a^{p_k}, hhat_a = (m_a/|Omega|)^{1/d} (eq. ViscMin)
  double relax[kMaxNloc];  // c_r * hhat_a^{p_r} (eq. ViscMinConst2)
  // Dirichlet data U^d of each box face (Dirichlet and supersonic kinds), and
  // its node fields as a node cache row holds them, written on the device at
  // set-up: U (dim+2), velocity (dim), p, a, p^-alpha, f(s), s~, 1/p
  double bstate[6][kMaxD + 2];
  double bnode[6][2 * kMaxD + 8];
  double xg[4];  // Gauss-Lobatto nodes on [0, 1] (node coordinates of time-dependent boundary data)
};

// Everything a kernel needs, passed by value.
struct KArgs {
  int64_t N, nblocks, ncells;
  int32_t R, W, nloc, nb1, deg, dim, cpb;
  int64_t cells[3];
  int32_t bc[6];
  int32_t bcdata;   // bit f: some part of face f has a data kind (Dirichlet, supersonic, in/outflow)
  // boundary parts with their own kinds (NULL: bc[f] everywhere): the kind of
  // the cell face with index idx over the other axes of face f at bcc[bcc_off[f] + idx]
  const int8_t *bcc;
  int64_t bcc_off[6];
  int32_t no_quiet; // GDG_FLAG_NO_QUIET_ROWS: sweep 2 marks no row quiet
  // data of the Dirichlet-type faces from the isentropic vortex (beta, x0,
  // u_inf, gamma) at the node and the stage time instead of bnode
  int32_t vortex_data;
  // data of the Dirichlet-type faces from U^n, the state at the start of the
  // step: its node records, written by the step's first stage
  int32_t old_data;
  double *Nold;
  double vx[6];
  double lo[3], hx[3];  // box corner and cell sizes (node coordinates)
  double gamma, cfl, c_ev, c_k, pk, c_r, p_r, vol;
  double alpha, inv_alpha;
  int32_t ipow;     // > 0: 1/alpha equals this integer, the p* power is taken by multiplies
  int32_t g75;      // gamma == 7/5: entropy comparisons by integer powers
  int32_t scheme, passes;
  // time integration: nst stages per step; stage k is a forward-Euler stage
  // of size tstep[k] * tau at time t + tfrac[k] * tau, and the first stage
  // picks tau = cfl * tau_max / tstep_max
  int32_t nst;
  double tstep[kMaxStages], tfrac[kMaxStages], tstep_max;
  int32_t mixed;    // 1: c_ij stored in FP32 and the flux / entropy-viscosity sums taken in FP32
  // Order in which the row blocks of a 3D mesh are swept (0: block order).
  // With whole x-lines of blocks, tiles of ty y-rows are swept z-plane by
  // z-plane, so the block one z-plane back was swept nbx * ty blocks earlier
  // (still in the XCD's L2) instead of a whole plane earlier.
  int32_t tiled;
  int64_t t_nbx, t_ny, t_nz, t_tx, t_ty;
  // stencil
  int32_t *col;
  double *c;        // dim planes of nslots (FP64 precision)
  float *cf;        // dim planes of nslots (mixed precision)
  uint8_t *meta;
  double *kscale;   // 1 / (kappa_i m_i) per row, kappa_i = 1/(card I(i) + 1)
  const RefTables *ref;
  // General (mapped) cells: the per-node and per-cell-class entries of ref
  // (mlump, hpk, relax, mblk, minv) are per row and per cell instead
  int32_t general;
  int32_t ustruct;      // unstructured: the host wrote col, meta and c (the fill kernel only sets boundary data)
  int32_t cg;           // continuous elements: rows are global nodes in blocks of R, no cell solve
  const double *mrow;   // m_i
  const double *hprow;  // c_k hhat_i^{p_k}
  const double *relrow; // c_r hhat_i^{p_r}
  const double *cmblk;  // per cell: m_ab (nloc x nloc)
  const double *cminv;  // per cell: (M_K^{-1})_ab
  int64_t nslots;
  // per-dof fields
  double *Nd;       // node records, two buffers of N * kNodeStride
  double *Qd;       // bound records (N * kQStride)
  double *Ld;       // limiter records (N * kLimStride)
  double *U1d;      // U^(1) records (N * kU1Stride)
  double *fsum;     // per row, (dim+2) planes: sum_j (f(U_j) - f(U_i)) c_ij with the boundary parts
  double *dL;       // d^L (and d^{d,L} on ghost slots) per slot
  double *l1;       // l of limiter pass 1 per slot (the ghost slot of a row holds l_i^d)
  uint8_t *accepted;  // per row: set by sweep 2 for rows of quiet cells (every flux zero), then by
                      // limiter pass 1: it accepted every flux of the row whole
  double *red;        // kRedBlocks * kRedFields partials of the state reduction, then kRedFields results
  unsigned long long *cnt;  // spread counters (kCntKinds * kCntSlots lines)
  Ctl *ctl;
};

// host-side entry points of the kernels (gdg_kernels.hip)
struct StageBufs {
  const double *in;   // stage input state
  double *out;        // stage output (may alias Un)
  const double *Un;   // the state the SSP combination takes (U^n, or a partial sum)
  double ca, cb;      // out = ca * Un + cb * Phi(in)
  // optional second output (NULL: none): out2 = cx * X2 + cy * Phi(in),
  // read and written at the same element (X2 may alias out2)
  double *out2;
  const double *X2;
  double cx, cy;
};
// Optional kernel timing: when a Prof is passed, each launch is bracketed by
// HIP events on the same stream (also inside a captured graph); the host folds
// them into per-kernel sums after the stream has synchronized.
enum { KID_PRIM = 0, KID_SWEEP1, KID_SWEEP2, KID_LIMIT1, KID_LIMIT2, KID_COUNT };
struct Prof {
  void **ev;      // hipEvent_t pairs, created by the host
  int *kid;       // kernel id of each bracketed launch
  int cap;        // capacity in launches
  int n;          // bracketed launches since the last harvest
};
// Work list of the request server: the resident requests of one class
// (dim, degree, precision), each with its kernel arguments and the buffers of
// the three SSP-RK3 stages, and the prefix sums of their row blocks.  The
// batched kernels walk all row blocks of all entries with one persistent grid,
// so a graph captured once serves every later mix of requests.
constexpr int kMaxBatch = 256;
struct BatchEntry {
  KArgs A;
  StageBufs sb[3];
};
struct BatchList {
  int32_t nreq;
  int32_t pad;
  int64_t ntiles;                      // sum of the entries' row blocks
  int64_t tile_begin[kMaxBatch + 1];   // first row block of each entry
  BatchEntry e[kMaxBatch];
};

bool build_ref_tables(int dim, int deg, const double *h, RefTables *T, std::string *err);

// Host tables of a mesh of general cells (gdg_mapped.cpp), for the row-blocked
// ELL layout of R rows per block and W slots per row.
struct MappedSetup {
  std::vector<double> mrow, hprow, relrow, kscale;  // per row
  std::vector<double> cmblk, cminv;                  // per cell, nloc x nloc
  std::vector<double> c;                             // dim planes of nslots, the slot order of the fill kernel
  double vol;                                        // |Omega|
  // unstructured meshes: the whole stencil (the fill kernel does not run)
  std::vector<int32_t> col;
  std::vector<uint8_t> meta;
};
bool build_mapped(const gdg_mesh_desc *m, const gdg_params *p, const double *vx, const RefTables &T, int R, int W,
                  int64_t nslots, MappedSetup *out, std::string *err);
// Continuous elements on the box (gdg_cg.cpp): per-row tables, c_ij, c_i^d
// and the whole ELL stencil (col, meta, c, kappa) for R rows per block and W
// slots per row.
bool build_cg(const gdg_mesh_desc *m, const gdg_params *p, int R, int W, int64_t nslots, MappedSetup *out,
              std::string *err);
// Node counts per axis of the continuous space of a box mesh.
void cg_nodes(const gdg_mesh_desc *m, int64_t *gn);
// Degree of the cell maps (1 multilinear, 2 quadratic) of a mesh of general cells.
int map_degree(const gdg_mesh_desc *m);
// Gauss-Legendre rule of n = 2 .. 5 points on [0, 1].
void gauss_rule01(int n, double *x, double *w);
// det J at xi of the degree-g map through a cell's points X, and its cofactor
// matrix cof = det(J) J^{-T}.
double map_jacobian(int d, int g, const double (*X)[3], const double *xi, double cof[3][3]);
// The (g+1)^dim points of cell K's map of degree g (point v: digits q_e of v
// in base g + 1, first axis lowest).
void mapped_cell_points(const gdg_mesh_desc *m, const double *vx, int64_t K, double (*X)[3]);
// x = F_K(xi) for the points X of a cell's map of degree g.
void mapped_point(int d, int g, const double (*X)[3], const double *xi, double *x);
int launch_fill(const KArgs &A, void *stream);
int launch_begin(const KArgs &A, double dt_cap, double tau_fixed, int device_driven, void *stream);
int launch_end(const KArgs &A, void *stream);
// the end of a device-driven step and the start of the next, in one launch
int launch_end_begin(const KArgs &A, void *stream);
int launch_set_run(const KArgs &A, double t_final, long long step_limit, void *stream);
// node records of the input of `stage` (of the current step) from the SoA state U
int launch_prim(const KArgs &A, const double *U, int stage, void *stream);
// min rho, min eps and sum_i m_i U_i (per component) of the state U into
// A.red[kRedBlocks * kRedFields ...], deterministically
int launch_state_stats(const KArgs &A, const double *U, void *stream);
// Zeroes the spread counters (a kernel, so that it may be captured).
int launch_zero_counts(const KArgs &A, void *stream);
// need_prim: launch the primitives sweep even when the last limiter pass of
// the previous stage wrote the node cache (the stage input was not produced by
// a completed stage of this context)
int launch_stage(const KArgs &A, const StageBufs &b, int stage, void *stream, Prof *prof, int need_prim);
// ksteps device-driven SSP-RK3 steps of every request in L (persistent grid of
// `grid` workgroups, a multiple of 8), then a copy of each request's control
// block into status[0 .. nreq).
int launch_batch_steps(int dim, int deg, int mixed, const BatchList *L, Ctl *status, int ksteps, int grid,
                       void *stream);

// Access to a context for the request server (gdg_api.cpp).
const KArgs &ctx_kargs(const gdg_ctx *ctx);
void ctx_stage_bufs(const gdg_ctx *ctx, StageBufs sb[3]);
// Arms the device-driven loop: run to t_final with no step limit, flags cleared.
int ctx_arm(gdg_ctx *ctx, double t_final);
// Takes the time and counters of a control block copied after device-driven steps.
void ctx_sync(gdg_ctx *ctx, const Ctl &c);
// Redoes the step that a CFL violation halted (host-driven, with the restart
// rule of gdg_step), then re-arms the device-driven loop.
gdg_status ctx_restart(gdg_ctx *ctx, const Ctl &c, double t_final);
const char *ctx_error(const gdg_ctx *ctx);
// Replays the context's captured graph of device-driven steps (captured at the
// first call) on `stream`; 0 on success.
int ctx_launch_steps(gdg_ctx *ctx, void *stream);
// The context's device control block.
const Ctl *ctx_dev_ctl(const gdg_ctx *ctx);
// The device-driven time loop of gdg_run_to(); use_graph = false enqueues
// the same launches directly instead of replaying a captured graph.
gdg_status run_loop(gdg_ctx *ctx, double t_final, int64_t max_steps, gdg_stats *stats, bool use_graph);
// Sets the text that gdg_last_error(NULL) returns on the calling thread.
void set_create_error(const std::string &msg);
// Time and step counters as the host last took them (no device work).
void ctx_counts(const gdg_ctx *ctx, double *t, int64_t *steps, int64_t *restarts);
// Status of a control block's bad_flag: GDG_E_BOUNDARY for bit 2 (subsonic
// flow at a supersonic face), else GDG_E_INADMISSIBLE with the text `what`;
// sets the context's error text.
gdg_status flag_status(gdg_ctx *ctx, int flag, const char *what);

}  // namespace gdg
