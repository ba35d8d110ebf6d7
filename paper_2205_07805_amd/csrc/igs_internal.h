// Internal types shared by the device kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace igs {

constexpr int kWave = 64;
constexpr int kReduceThreads = 512;     // 8 waves per block in the fused reduction
constexpr int kReduceWaves = kReduceThreads / kWave;
constexpr int kUpdateThreads = 256;
constexpr int kUpdateRows = 4;          // rows per thread in the update / x-update passes
constexpr int kMaxBlocks = 2048;        // most blocks of a kernel that writes partial sums
constexpr long long kGemvLdsMax = 8192;   // most columns (lda) of the shared-memory dense kernel
constexpr int kMaxGroups = 64;          // rows of the group-partial buffer (8 are used; the rest
                                        // is scratch for the explicit-norm fallback)

// How a restart cycle ended (mirrors IGS_CYCLE_* in igs.h).
enum CycleStatus : int {
  kRunning = 0, kConvStart = 1, kConverged = 2, kFull = 3,
  kBreakdown = 4, kLagnorm = 5, kMaxit = 6, kNonfinite = 7
};

// What the update kernel of an iteration does.
enum UpdateMode : int {
  kUpdNone = 0,      // nothing (cycle ended without needing v_j)
  kUpdNormal = 1,    // v_j and u_{j+1}
  kUpdVOnly = 2,     // v_j only (last vector of a cycle, on request)
  kUpdFallback = 3,  // lagged norm cancelled: w = u - V t, explicit ||w||, finish column
  kUpdCorrect = 4    // two-reduce second sweep: w = u - V t in place, t = T r2
};

// Control block in device memory.  Written by block 0 of the update kernel
// (and by the last block of the explicit-norm fallback); read at the start of
// every step kernel so that kernels queued after the end of a cycle do
// nothing.  end_iter is the iteration at which the cycle ended: a kernel of
// iteration j runs only while end_iter >= j, so the other blocks of the
// kernel that ends the cycle still do their share.
constexpr int kNotEnded = 1 << 30;

struct Ctl {
  int end_iter;        // kNotEnded while the current cycle runs
  int J;               // finished Hessenberg columns in the current cycle
  int status;          // CycleStatus
  int mode;            // UpdateMode of iteration mode_iter (as decided by block 0)
  int mode_iter;       // iteration the mode applies to (-1: none)
  int breakdowns;
  int fallbacks;
  int gs;              // 1 or 2 Gauss-Seidel sweeps
  int final_v;
  int m;               // restart length of the cycle
  long long n;
  long long its_before;  // iterations finished before this cycle
  long long maxit;
  double bnorm;        // ||b||
  double tol;          // relative tolerance
  double tol_abs;      // tol * ||b||
  double lagnorm_tau;
  double rho;          // ||r0|| of the cycle
  double gabs;         // |g_J| after the last finished column
  double gamma_prev;   // gamma of the previous iteration
  double cycle_rtol;   // > 0: a cycle also ends once |g_j| <= cycle_rtol * rho
  double tol_cyc;      // the Arnoldi-residual target of the current cycle
  int nonfinite_in;    // count of non-finite entries in b and x0
  int pad;
};

// Device operator: CSR or dense row-major.
struct Op {
  int dense;
  long long n;
  const int* row_ptr;
  const int* col_idx;
  const double* vals;
  const double* A;     // dense (columns n..lda-1 of every row hold zeros)
  long long lda;
  int dense_mfma;      // dense: 0 = one wave per row, 1 = the matrix cores,
                       // 2 = x staged in shared memory (lda <= kGemvLdsMax)
  int lpr;             // CSR lanes per row
  const float* vals32; // CSR values rounded to FP32 (mixed precision; may be null)
  int rpg;             // CSR rows per lane group (0: the default for lpr; set by the tuner)
  // The same matrix in column-major ELL form (rows of at most 8 entries,
  // lpr == 8): entry k of row r at k * n + r, padded with (column 0, value
  // 0); ell_k = 0 when absent.  Its product is bit-identical to the CSR one.
  int ell_k;
  const int* ell_col;
  const double* ell_val;
  const float* ell_val32;
  // The ELL column indices as 16-bit offsets from the row (col - r; padding
  // 0, with value 0), when every entry lies within 32,767 columns of its
  // row; null otherwise.  The fused operator apply reads these (10 bytes per
  // FP64 entry instead of 12); the products are the ELL form's, with padding
  // multiplying x[r] instead of x[0] (both by zero).
  const short* ell_dcol;
};

// Device workspace of a context (all device pointers).
struct Work {
  double* V; long long ldv;      // basis, column-major, m+1 columns
  double* z;                     // A u of the current iteration
  double* H;                     // Hessenberg before rotation, packed by columns (m(m+3)/2)
  double* R;                     // rotated Hessenberg, column-major, ld = ldh
  double* T;                     // (I + L)^{-1}, packed lower triangle by rows ((m+1)(m+2)/2)
  double* L;                     // strictly lower L, column-major, ld = ldt
  int ldh; int ldt;
  double* cs; double* sn; double* g; double* y;
  double* coef_t;                // t of the current iteration (prev at the next)
  double* coef_r1;               // r1 of the current iteration (prev at the next)
  double* part;                  // per-block partial sums [kMaxBlocks][pstride]
  double* gpart;                 // per-group partial sums [kMaxGroups][pstride]
  int pstride;
  unsigned* tickets;             // [kMaxGroups + 1] arrival counters
  Ctl* ctl;
  float* V32;                    // FP32 basis (mixed precision), same ldv
  float* z32;                    // FP32 A u
  int fp32;                      // 1: the step kernels work on V32 / z32
  // Host memory, read by the launchers only (null: the default grids): for
  // iteration j, bit 0 halves the blocks of the fused reduction and bit 1
  // those of the update (each block then takes twice the rows).
  const unsigned char* tune;
  // The small products of an iteration whose T and H do not fit the update
  // kernel's shared memory, formed beforehand by coef_kernel (3 (m + 2)
  // doubles); pre_on = 0: every update block forms them itself.
  double* pre;
  int pre_on;
  // 1: a small system's update may split the columns of a tile over the
  // waves of a block (per-row sums then run over four quarters of the
  // columns).  Off where results must match the batched kernels bit for bit,
  // whose row sums run over the columns in order: on for dense operators
  // only, which are never batched.
  int col_split;
  // The fused reduction's column split of the current launch (set by its
  // launcher; <= 1: none).
  int red_csplit;
};

// Groups of the first level of the deterministic grid reduction for a grid
// of nb blocks (blocks b with the same b % 8 form a group).
__host__ __device__ inline int reduce_groups(int nb) { return nb < 8 ? nb : 8; }

// ---- launchers (kernels.hip) ------------------------------------------------

// gate: skip when the cycle ended before iteration j (nullptr: always run).
hipError_t launch_spmv(const Op& op, const double* u, double* z, const Ctl* gate, int j,
                       hipStream_t s);
// Cycle start: reset the control block, then r = b - A x (FP64) into column 0
// (its_before < 0: keep the value the host wrote into the control block)
// of the basis (V, or V32 rounded to FP32 when w.fp32).
hipError_t launch_residual(const Op& op, const double* b, const double* x, const Work& w,
                           long long its_before, long long maxit, int m, int gs, int final_v,
                           double tol, double tau, double cycle_rtol, hipStream_t s);
hipError_t launch_spmv32(const Op& op, const float* u, float* z, const Ctl* gate, int j,
                         hipStream_t s);
hipError_t launch_round_to_float(const double* src, float* dst, long long count, hipStream_t s);
// The column-major ELL form of a CSR operator with rows of at most K <= 8
// entries (device arrays; ec, ev hold K n entries).
hipError_t launch_csr_to_ell(long long n, int K, const int* rp, const int* ci, const double* va,
                             int* ec, double* ev, hipStream_t s);
hipError_t launch_bnorm(const double* b, const double* x, long long n, const Work& w,
                        hipStream_t s);
hipError_t launch_reduce(const Work& w, long long n, int j, bool with_z, hipStream_t s,
                         int* nblocks_out);
// The operator apply fused into the reduction (z = A u_j for each block's own
// rows, then the reduction with z from shared memory; z is also stored for
// the update).  opreduce_fits: whether iteration j can take it (an ELL form,
// n a multiple of 4, aligned arrays, a block's rows of z within its shared
// memory); otherwise launch_spmv* and launch_reduce run as two kernels.  The
// results are bit-identical either way.
bool opreduce_fits(const Op& op, const Work& w, long long n, int j);
hipError_t launch_opreduce(const Op& op, const Work& w, long long n, int j, hipStream_t s,
                           int* nblocks_out);
// Whether iteration j's small products run in a kernel of their own before
// the update (w.pre_on, and T and H beyond the update's shared memory).
bool coef_kernel_needed(const Work& w, int j);
// That kernel: t = T p (or T q / gamma with one sweep), H (t_prev / gamma_prev)
// and the new row of T, one wave per output.
hipError_t launch_coef(const Work& w, int j, int ngroups, hipStream_t s);
// ngroups: the group totals the reduction of iteration j left in w.gpart.
hipError_t launch_update(const Work& w, long long n, int j, int gs, int ngroups, hipStream_t s);
// Second Gauss-Seidel sweep of the two-reduce variant for the vector in
// column j (after the reduction of [V_{0:j}, u]^T u): r2 = V_{0:j}^T u,
// r3 = (I + L_{0:j})^{-1} r2, u -= V_{0:j} r3 in place, and r3 is added to
// the stored first-sweep coefficients of column j-1.
hipError_t launch_correct(const Work& w, long long n, int j, int ngroups, hipStream_t s);
hipError_t launch_lsq(const Work& w, int m, hipStream_t s);
hipError_t launch_xupdate(const Work& w, long long n, double* x, hipStream_t s);

// Modified Gram-Schmidt comparator (FP64): ||r0|| and v_0 = r0 / ||r0||;
// then, after z = A v_c has been written to V[:, c+1], the c + 2 reductions
// of column c and v_{c+1}.
constexpr int kMgsMaxCols = 512;       // most columns of a cycle (the largest restart)
hipError_t launch_mgs_start(const Work& w, long long n, hipStream_t s);
hipError_t launch_mgs_column(const Work& w, long long n, int c, hipStream_t s);

// Step kernels on caller buffers (no control block).
hipError_t launch_reduce_raw(const double* V, long long ldv, long long n, int j, const double* z,
                             double* part, double* gpart, int pstride, unsigned* tickets,
                             double* out, hipStream_t s);
// The same reduction with its partial sums and counters in the library's
// static device array (no allocation; calls overlapping on one device race).
// Columns j + 1 <= kNoAllocMaxCols; out: device, 2 (j + 1) doubles.
constexpr int kNoAllocMaxCols = 256;
constexpr size_t kNoAllocBytes =
    ((size_t)(kMaxBlocks + kMaxGroups) * 2 * kNoAllocMaxCols + 64) * sizeof(double);
hipError_t launch_reduce_noalloc(const double* V, long long ldv, long long n, int j,
                                 const double* z, double* out, hipStream_t s);
hipError_t launch_update_raw(double* V, long long ldv, long long n, int j, const double* z,
                             const double* t, const double* r1, double inv_gamma, hipStream_t s);

// ---- batches: many independent solves advanced together --------------------
//
// Every launch of a batched step runs the same step for all instances of a
// batch: instance k gets a contiguous range of the grid (starting at a
// multiple of 8, so block k mod 8 still names its XCD) and sees it as a grid
// of its own.  Each instance's grid, and so its summation order, is the one a
// lone solve of that instance would launch, which keeps every result
// bit-identical to the lone solve.

constexpr int kMaxBatch = 32;

// One instance of a batch (device table, written by the host once per cycle).
struct Inst {
  Work w;              // its workspace and control block
  Op op;               // its CSR operator
  long long n;
  const double* b;
  double* x;
  long long its_before;  // iterations finished before this cycle
  long long maxit;       // iteration budget of this cycle
  double tol, tau, cycle_rtol;
  int m, gs, final_v;
  int run_lsq;           // 0: the cycle is a final check (iteration 0 only)
};

// Host view of a batch for one launch: the instances taking part.
struct BatchRun {
  const Inst* d_tab;   // device table
  const Inst* h_tab;   // its host copy (sizes and operators)
  int act[kMaxBatch];  // table rows taking part
  int count;
  hipStream_t stream;
  int reduce_rows;     // least rows per block of the fused reduction (1: lone grid)
  int update_tiles;    // least tiles per block of the update (1: lone grid)
};

// ||b|| and the finiteness check of the instances act[0..count).
hipError_t batch_bnorm(const BatchRun& r);
// Cycle start: reset each control block, then r = b - A x into column 0.
hipError_t batch_residual(const BatchRun& r);
// z = A u_j for every instance (skipped per instance once its cycle ended).
hipError_t batch_spmv(const BatchRun& r, int j);
// The fused reduction of iteration j; ngroups[k] receives the group count
// of instance act[k] for the update.
hipError_t batch_reduce(const BatchRun& r, int j, bool with_z, int* ngroups);
hipError_t batch_update(const BatchRun& r, int j, const int* ngroups);
// R y = g and x += V y for the instances with run_lsq.
hipError_t batch_lsq(const BatchRun& r, int m);
hipError_t batch_xupdate(const BatchRun& r);
// Copy each instance's control block to out[act[k]] (device memory).
hipError_t batch_ctl_gather(const BatchRun& r, Ctl* out);

}  // namespace igs
