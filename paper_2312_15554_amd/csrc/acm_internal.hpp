// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acm {

// Geometry of one periodic cell.  Real fields: [comp][z][y][x], x fastest.
// Half spectra (after the x real-to-complex pass): [comp][z][y][xh] with
// xh = nx/2 + 1.  For dim == 2, nz == 1 and the "last axis" is y.
struct Geom {
  int dim;
  int nx, ny, nz;
  int xh;            // nx/2 + 1
  int64_t ntot;      // nx*ny*nz
  int64_t nrows;     // ny*nz  (x rows per component)
  int64_t nspec;     // nz*ny*xh complex values per component
  int last_n;        // length of the last axis (nz in 3D, ny in 2D)
  int64_t plane;     // complex values per index of the last axis (ny*xh in 3D, xh in 2D)
};

// Per-cell device tables (working precision T): FFT twiddles for the three
// lengths used (nx/2, ny, nz), the real-transform twiddles W^k = exp(-2 pi i k/nx)
// for k in [0, nx/2], and the per-axis derivative symbols
// s(m) = sin(2 pi m/n)/h and l(m) = 4 sin^2(pi m/n)/h^2.
struct TableOffsets {
  int tw_x;    // complex offsets into the complex table
  int tw_y;
  int tw_z;
  int rtw;
  int ncomplex;
  int sx, lx, sy, ly, sz, lz;  // real offsets into the real table
  int nreal;
};

// ADMM state that changes every iteration.  A solve keeps two slots: the
// passes of iteration n read slot n mod 2 and Step 4 of iteration n writes
// slot (n + 1) mod 2, so no pass ever reads a slot that the same launch is
// writing.  The parity is a kernel argument.
struct StokesState {
  double psi[3];      // alpha, beta, b of the iteration that reads this slot
  double c_prev;      // b/(b+alpha) of the iteration before it
  double rp[3], rd[3], tp[3], td[3], mu[3];  // residuals of the iteration that wrote it
  double s_min;       // smallest sum of the six residuals so far (divergence test)
  int64_t iter;       // iterations completed
  int32_t done;       // sticky: once set in either slot every pass exits at once
  int32_t status;     // 0 ok, 1 not converged, -5 diverged
  // Step 1 of the iteration that reads this slot is in increment form: the
  // spectra hold X = rhs^n - M u^n (the change of the right-hand side since
  // the last solve), the green pass solves M du = X and the local pass adds du
  // to u.  Otherwise they hold r and Step 1 is solved for u itself.
  int32_t incr;
  int32_t pad_;
};

// Device control block for one ADMM solve: constant parameters written by the
// host, the two state slots, and the words of the cross-workgroup protocols.
struct StokesCtl {
  double phi[3], tau[3], psi_min[3];
  double eps;
  double sqrt_n[3];   // sqrt(d N), sqrt(N), sqrt(d N)
  double nu;
  double g[3];
  int64_t max_iter;
  int32_t adaptive;
  int32_t hist_cap;   // capacity of the residual history ring (entries)
  int32_t fault;      // non-zero: a single-launch slab pass gave up at its gate
  // non-zero (1 + state slot): the Step 4 kernel of pass mode 4 found b
  // changed; every pass after it skips until the host has formed r again
  int32_t hold;
  // the local passes form X (increment form) for the next Step 1; Step 4 keeps
  // that form while b is unchanged (a change of b makes the rhs pass form r)
  int32_t incr_enabled;
  int32_t pad_;
  StokesState st[2];
  // Words that many workgroups hit at once sit on cache lines of their own,
  // away from the parameters every workgroup reads when it starts.
  alignas(256) uint32_t counter;  // workgroups of a local pass that have finished
  alignas(256) uint32_t gate;     // single-launch slab pass: gate generations
};

__host__ __device__ inline bool stokes_done(const StokesCtl* c) {
  return (c->st[0].done | c->st[1].done) != 0;
}
// a pass of the solve has nothing to do: it stopped, or it is held
__host__ __device__ inline bool stokes_skip(const StokesCtl* c) {
  return (c->st[0].done | c->st[1].done | c->hold) != 0;
}

// Iterations in the paper's form before the increment form of Step 1 may
// start (see StokesState::incr).
constexpr int64_t kIncrAfter = 64;

// One history record per iteration: rp[3], rd[3], tp[3], td[3], psi[3].
constexpr int kHistDoubles = 15;

// Kernel timing in the profiling mode: when the calling thread's
// launch_events() holds two events, the next kernel launched through
// ACM_LAUNCH records the start and end of its own execution in them (the
// dispatch's timestamps, no stream commands in between) and clears them.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
LaunchEvents& launch_events();

// Control block for one Lippmann-Schwinger solve (one time step at a time).
// Per-iteration LS state, two slots chosen by iteration parity (as for the
// ADMM state): the passes of iteration n read slot n mod 2 and the stop test
// that follows writes slot (n + 1) mod 2.
struct TransportState {
  double r1, r2;
  double r1_min;        // smallest r_1 of the current time step (divergence test)
  int64_t iter;         // iterations in the current time step
  int64_t total_iter;
  int32_t done;         // sticky: once set in either slot every pass exits
  int32_t status;
  int32_t pend;         // slab path: a green pass ran whose partials are not yet judged
  int32_t pad_;
};

struct TransportCtl {
  double eps;
  double sqrt_n1, sqrt_n2;
  double inv_dt;        // 0 for the steady cell problem
  double A0, B0[3];
  double g[3];
  double Pe, eta, diff;
  double calF;          // Pe * ubar . g  (multiplied by (1-H) per voxel)
  int64_t max_iter;
  int32_t steady;
  int32_t flux;         // flux form of the diffusive term (face harmonic means, D+ / D-)
  TransportState st[2];
  alignas(256) uint32_t counter;  // on its own cache line (see StokesCtl)
};

__host__ __device__ inline bool transport_done(const TransportCtl* c) {
  return (c->st[0].done | c->st[1].done) != 0;
}

// Stop test of eq. tol_solute from the Parseval totals of one green pass (the
// divergence guard included): the state after `cur`.
__host__ __device__ inline TransportState transport_judge(const TransportCtl* c,
                                                          const TransportState& cur,
                                                          double tot0, double tot1,
                                                          int64_t ntot) {
  TransportState nx = cur;
  const double inv_n = 1.0 / (double)ntot;
  const double r1 = sqrt(tot0 * inv_n), r2 = sqrt(tot1 * inv_n);
  nx.r1 = r1;
  nx.r2 = r2;
  nx.iter = cur.iter + 1;
  nx.total_iter = cur.total_iter + 1;
  nx.pend = 0;
  // divergence: non-finite, or r_1 grown a millionfold over its minimum
  // (the LS iteration contracts only for a large enough comparison medium)
  if (r1 < nx.r1_min) nx.r1_min = r1;
  if (!isfinite(r1) || !isfinite(r2) || (nx.iter > 5 && r1 > 1e6 * nx.r1_min)) {
    nx.done = 1;
    nx.status = -5;
  } else if (r1 <= c->sqrt_n1 * c->eps && r2 <= c->sqrt_n2 * c->eps) {
    nx.done = 1;
    nx.status = 0;
  } else if (nx.iter >= c->max_iter) {
    nx.done = 1;
    nx.status = 1;
  }
  return nx;
}

// Per-cell device pointers of one Stokes solve.  Kernels of a batched launch
// read the entry of their cell (blockIdx.z); a single cell passes it by value.
struct StokesCellArgs {
  void* spec;          // complex [d][nspec]
  void* qhat;          // complex [nspec]
  void* dhat;          // complex [nspec]
  void* u;             // real [d][ntot]
  void* a;             // real [d][ntot]
  const uint8_t* H;    // uint8 [ntot]
  double* part;        // green partials [3*ngreen]
  double* lpart;       // local partials: [4*nlocal] (rows, single launch) or [7*nlocal] (slabs)
  StokesCtl* ctl;
  double* hist;        // may be null
};

// Per-cell pointers of a column (y or z) transform.
struct ColCellArgs {
  void* data;
  const int32_t* skip;   // may be null; when *skip != 0 the cell is skipped
  const int32_t* skip2;  // a second such flag (the other state slot), may be null
};

enum KernelKind {
  KK_GREEN = 0,
  KK_LOCAL = 1,
  KK_RHS = 2,
  KK_YINV = 3,
  KK_YFWD = 4,
  KK_T_GREEN = 5,
  KK_T_LOCAL = 6,
  KK_OTHER = 7,
  KK_COUNT = 8
};

// ----------------------------------------------------------------- launchers
// All return hipSuccess or an error; an unsupported length returns
// hipErrorInvalidValue.

template <typename T>
struct DevTables {
  const void* ctab;  // cplx<T>[ncomplex]
  const T* rtab;     // T[nreal]
  TableOffsets off;
};

bool fft_length_supported(int n);

// Plain transforms (utility; init and readout).
template <typename T>
hipError_t launch_rows_r2c(const Geom& g, const DevTables<T>& tb, int nfields, const T* in,
                           void* out, hipStream_t s);
template <typename T>
hipError_t launch_rows_c2r(const Geom& g, const DevTables<T>& tb, int nfields, const void* in,
                           T* out, double scale, hipStream_t s);
// Complex transform along y (axis 1) or z (axis 2) of nfields half spectra, in place.
// `skip`, `skip2` (each may be null): device flags; when either is non-zero the
// launch does nothing.
template <typename T>
hipError_t launch_cols(const Geom& g, const DevTables<T>& tb, int axis, int sign, int nfields,
                       void* data, hipStream_t s, const int32_t* skip = nullptr,
                       const int32_t* skip2 = nullptr);
// Batched form: cells[0..ncells) (device array) with one transform each.
template <typename T>
hipError_t launch_cols_batched(const Geom& g, const DevTables<T>& tb, int axis, int sign,
                               int nfields, const ColCellArgs* cells, int ncells, hipStream_t s);

// Stokes ADMM passes.  `one` is used when `many` is null (single cell);
// otherwise cell i = blockIdx.z reads many[i] and ncells cells are launched.
// `variant` 0, 1, 2: LDS-staged kernel with tile width per ColCfg; 3, 4:
// register-resident kernel with the tile widths of 0 and 1; 5, 6: LDS-staged
// kernel with one thread group per field during the transforms, tile widths
// of 0 and 1 (kGreenVariants in all); *nblocks receives
// the number of workgroups per cell (= partial-sum records written).
constexpr int kGreenVariants = 7;
// rounds in which the autotuner times every green variant (best round kept)
constexpr int kTuneRounds = 3;
// iterations of a pass-mode-4 solve that form Step 4 in the rhs pass before
// the Step 4 kernel takes it over (Step 4 changes b in most of the first few
// dozen)
constexpr int64_t kRhsStep4Iters = 64;

// `par`: parity of the iteration (the state slot its passes read).  The row
// local pass runs Step 4 in its last workgroup and writes slot par ^ 1; the row
// rhs pass reads the slot given as `slot` (par ^ 1 within the iteration, the
// initial slot for the right-hand side of a warm start).
template <typename T>
hipError_t launch_stokes_green(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                               const StokesCellArgs* many, int ncells, int par, int variant,
                               int* nblocks, hipStream_t s);
template <typename T>
hipError_t launch_stokes_local(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                               const StokesCellArgs* many, int ncells, int par, int green_blocks,
                               hipStream_t s);
template <typename T>
hipError_t launch_stokes_rhs(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                             const StokesCellArgs* many, int ncells, int slot, hipStream_t s);

// Lippmann-Schwinger passes.  mode 0: LS update; mode 1: grad chi-hat only.
// `par`: iteration parity.  judge = 1: the last workgroup applies the stop
// test (writes slot par ^ 1); judge = 0: only the partial sums are posted and
// the next slab pass judges them.
// flux = 1: flux form (row input form only; see k_transport_green).
template <typename T>
hipError_t launch_transport_green(const Geom& g, const DevTables<T>& tb, int mode, void* spec,
                                  void* chat, const void* chat_m, double* partials,
                                  TransportCtl* ctl, int slab, int par, int judge,
                                  hipStream_t s, int flux = 0);
// Slab form of the local pass (3D, nx == ny <= 128, u 16-byte aligned): reads
// grad chi-hat from fields 0..2 and writes G_x, G_y, f_z (fields 0..2) and
// tau_z (field 3) for the green pass's slab input form (slab = 1).
// Every workgroup first judges the pending green pass from its partial sums
// (slot par; workgroup 0 stores the result in slot par ^ 1), then runs the
// local pass unless the solve has stopped.
template <typename T>
hipError_t launch_transport_slab(const Geom& g, const DevTables<T>& tb, void* spec, const T* u,
                                 const uint8_t* H, TransportCtl* ctl, const double* partials,
                                 int ngreen, int par, hipStream_t s);
template <typename T>
hipError_t launch_transport_local(const Geom& g, const DevTables<T>& tb, void* spec, const T* u,
                                  const uint8_t* H, const TransportCtl* ctl, hipStream_t s,
                                  int flux = 0);
// Green workgroups per cell (= partial-sum records) for the row (slab = false)
// or slab input form, or the flux form (row input form).
int transport_green_blocks(const Geom& g, int precision_bytes, bool slab, bool flux = false);

// FP64 reductions (per-block partials; the host adds them in order).
template <typename T>
hipError_t launch_flow_sums(const Geom& g, const T* u, const uint8_t* H, double* part, int* nsums,
                            hipStream_t s);
template <typename T>
hipError_t launch_chi_sums(const Geom& g, const T* chi, const T* u, const uint8_t* H,
                           double* part, int* nsums, hipStream_t s);
int reduction_blocks(const Geom& g);
// Upper bound of reduction_blocks() over every grid.
constexpr int kReductionBlocksMax = 512;
// Largest number of partial sums per block record (k_chi_sums in 3D: 8).
constexpr int kReductionSumsMax = 8;
// out[k] = sum over b in [0, nb) of part[b * ns + k], added in block order from
// 0.0 (one workgroup); ns <= 64.
hipError_t launch_sum_partials(const double* part, int nb, int ns, double* out, hipStream_t s);

// Warm start: a = H (g - grad q + nu Delta_h u0), div = div_c u0 (real, in
// `div`), then u <- (1-H) u in place.  q may be null (q0 = 0).
template <typename T>
hipError_t launch_warm_init(const Geom& g, const T* u, const T* q, const uint8_t* H, T* a, T* div,
                            double nu, const double* gp, hipStream_t s);

// An empty kernel (profiling: calibrates the per-launch event overhead).
hipError_t launch_noop(hipStream_t s);

// Row-step pass structure (single cell): rows_step (inverse x transform,
// Steps 2-3, next right-hand side with the b of the iteration, forward x
// transform, one record per workgroup), the Step 4 kernel without the hold
// word, and rows_rhs_cond (r again from u, a and H only when Step 4 changed b).
int rows_step_blocks(const Geom& g, int prec_bytes);
template <typename T>
hipError_t launch_rows_step(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                            int par, int green_blocks, hipStream_t s);
template <typename T>
hipError_t launch_rows_rhs_cond(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                                int par, hipStream_t s);
hipError_t launch_step4_nohold(const Geom& g, const StokesCellArgs& one, int par, int nrec,
                               hipStream_t s);

// Fused xy-slab Stokes passes (3D, nx == ny, slab of one field in LDS).
template <typename T>
bool slab_supported(const Geom& g);
template <typename T>
int slab_local_blocks(const Geom& g);
// The slab local pass only posts its partial sums; every workgroup of the
// slab rhs pass then forms Step 4 itself from all partials (the same bits in
// each), and workgroup 0 stores the new state in slot par ^ 1 (step4 = 1).
// With step4 = 0 the rhs pass uses slot par as it is (warm-start set-up).
template <typename T>
hipError_t launch_slab_local(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                             const StokesCellArgs* many, int ncells, int par, int green_blocks,
                             hipStream_t s);
template <typename T>
hipError_t launch_slab_rhs(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                           const StokesCellArgs* many, int ncells, int par, int step4,
                           int green_blocks, hipStream_t s);
// Step 4 of one cell from the records of the slab local pass, in one
// workgroup: slot par ^ 1 and the history record are written, and the hold
// word is set (1 + (par ^ 1)) when Step 4 changed b.  Pass mode 4 runs it in
// place of the rhs pass, whose r the slab local pass has formed with the old b.
template <typename T>
hipError_t launch_slab_step4(const Geom& g, const StokesCellArgs& one, int par, int nrec,
                             hipStream_t s);
// Local and rhs slab passes of one cell in a single launch: every workgroup
// runs the local pass, waits at a device-wide gate that the last one opens
// after Step 4, then runs the rhs pass on the slab still held in LDS.  Valid
// only when all nz * dim workgroups can be resident at once on the current
// device: slab_fused_capacity() returns how many can (0 if unsupported).
template <typename T>
int slab_fused_capacity(const Geom& g);
template <typename T>
hipError_t launch_slab_fused(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                             int par, int green_blocks, hipStream_t s);

// FNO kernels (k_fno.hip).
hipError_t fno_lift(const uint8_t* H, const uint16_t* Pw, const uint16_t* Pb, float* v, int C,
                    int64_t nvox, int B, hipStream_t s);
hipError_t fno_gather(const void* spec, void* out, const int* midx, int nm, int64_t nspec,
                      int nfields, hipStream_t s);
hipError_t fno_mix(const void* Xm, const uint16_t* R, void* spec, const int* midx, int nm, int C,
                   int B, int64_t nspec, bool adjoint, hipStream_t s);
hipError_t fno_dR(const void* Fm, const void* Xm, const float* mw, float* dR, int nm, int C,
                  int B, float inv_n, hipStream_t s);
hipError_t fno_pointwise(int C, const float* vin, const float* k, const uint16_t* W,
                         const uint16_t* b, float* pre, float* vout, int64_t nvox, int B,
                         int act, hipStream_t s);
hipError_t fno_pointwise_bwd(int C, const float* dv, const float* pre, const uint16_t* W,
                             float* dpre, float* dvdir, int64_t nvox, int B, int act,
                             hipStream_t s);
hipError_t fno_add(float* a, const float* b, int64_t n, hipStream_t s);
hipError_t fno_project(int C, const float* v, const uint16_t* Q1, const uint16_t* c1,
                       const uint16_t* Q2, const uint16_t* c2, float* out, int Cp, int64_t nvox,
                       int B, hipStream_t s);
hipError_t fno_project_bwd(int C, const float* v, const float* dout, const uint16_t* Q1,
                           const uint16_t* c1, const uint16_t* Q2, float* h, float* dh, float* dv,
                           int Cp, int64_t nvox, int B, hipStream_t s);
int fno_outer_blocks(int64_t nvox, int B);
hipError_t fno_outer(const float* A, const float* Bm, const uint8_t* Bu8, int P, int Q,
                     int64_t nvox, int B, float* part, float* out, hipStream_t s);
hipError_t fno_adam(float* p, uint16_t* pb, const float* g, float* m, float* v, int64_t n,
                    float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t fno_to_bf16(const float* p, uint16_t* pb, int64_t n, hipStream_t s);
hipError_t fno_mse(const float* out, const float* tgt, float* dout, int64_t n, double inv_count,
                   double* part, int nblk, hipStream_t s);

// Grid-size helpers used by the host to size partial-sum buffers.
int stokes_green_blocks(const Geom& g, int precision_bytes, int variant);
int stokes_local_blocks(const Geom& g, int precision_bytes);

}  // namespace acm
