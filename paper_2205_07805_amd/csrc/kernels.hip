// gfx950 kernels of the one-reduction Arnoldi step of iterated Gauss-Seidel GMRES.
//
// Per Arnoldi iteration j (0-based; iteration j normalises basis vector j and
// finishes Hessenberg column j-1) the host queues three kernels:
//
//   spmv     z = A u_j                              (operator apply; skipped at j = m)
//   reduce   [V_{0:j}, u_j]^T [u_j, z]              (the ONE global reduction;
//                                                     it ends with 8 group totals)
//   update   in every block: the totals, then the small solve (lagged norm,
//              second Gauss-Seidel sweep, Stephen's trick; block 0 also the
//              Hessenberg column, Givens rotation, rows of L and T, stopping
//              tests), then its share of
//            v_j = (u_j - V t) / gamma,
//            u_{j+1} = z / gamma - V r1 - v_j r1_j     (one pass over V)
//
// u_j lives in column j of V until the update overwrites it with v_j.  All
// reductions are deterministic: every partial sum is formed in a fixed order
// that depends only on the launch shape.
#include "igs_internal.h"

#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace igs {

constexpr int LPR_RPG_MAX = 4;  // rows per lane group for rows of <= 8 lanes

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Cross-lane sums with DPP moves (register to register, no LDS round trip).
// A double moves as its two 32-bit halves.  dpp_ctrl values (GFX9 encoding):
// quad_perm [1,0,3,2] = 0xB1 and [2,3,0,1] = 0x4E exchange lanes i^1 and i^2
// inside each group of 4; row_half_mirror = 0x141 maps lane i to 7-i inside
// each group of 8; row_mirror = 0x140 maps lane i to 15-i inside each row of
// 16.  After the steps up to a group size every lane of the group holds the
// group's sum, added in the same order in every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16); every lane of a
// group gets the group's sum.  All lanes of the wave must be active.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_move<0xB1>(v);
  if constexpr (G >= 4) v += dpp_move<0x4E>(v);
  if constexpr (G >= 8) v += dpp_move<0x141>(v);
  if constexpr (G >= 16) v += dpp_move<0x140>(v);
  return v;
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_move<0xB1>(v);
  if constexpr (G >= 4) v += dpp_move<0x4E>(v);
  if constexpr (G >= 8) v += dpp_move<0x141>(v);
  if constexpr (G >= 16) v += dpp_move<0x140>(v);
  return v;
}

// Sum over the 64 lanes of a wave, returned in every lane (a wave-uniform
// value).  All lanes of the wave must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v = group_sum<16>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Two consecutive rows of a column as one 16-byte access.
typedef double dvec2 __attribute__((ext_vector_type(2)));

// Streaming read of data used once per kernel (the basis V): non-temporal,
// so it does not displace reused data from the caches.
__device__ __forceinline__ dvec2 ld_stream2(const double* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
}
__device__ __forceinline__ dvec2 ld2(const double* p) { return *reinterpret_cast<const dvec2*>(p); }

// 16-byte vectors of the basis element type: W consecutive rows per lane
// (2 doubles or 4 floats).
template <typename T> struct Vec16;
template <> struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};
template <> struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <typename T>
__device__ __forceinline__ typename Vec16<T>::type ld16(const T* p) {
  return *reinterpret_cast<const typename Vec16<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ typename Vec16<T>::type ld16_stream(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const typename Vec16<T>::type*>(p));
}
// Non-temporal 16-byte store: the basis update's outputs.  The next kernels
// read these vectors once; stored this way, the fused reduction that first
// reads them runs faster (0.5% on the whole 2M-row solve, 1% with the
// operator apply storing z the same way).
template <typename T>
__device__ __forceinline__ void st16(T* p, const typename Vec16<T>::type& v) {
  __builtin_nontemporal_store(v, reinterpret_cast<typename Vec16<T>::type*>(p));
}

__device__ __forceinline__ int load_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Does iteration j of the current cycle run (the cycle has not ended before it)?
__device__ __forceinline__ bool ctl_runs(const Ctl* c, int j) { return load_agent(&c->end_iter) >= j; }

// The blocks of one operation as its code sees them: block `bid` of `nb`.
// A kernel that runs one instance uses (blockIdx.x, gridDim.x); a batched
// kernel gives each instance a contiguous range of its grid.
struct Grid {
  int bid;
  int nb;
};
__device__ __forceinline__ Grid hw_grid() { return Grid{(int)blockIdx.x, (int)gridDim.x}; }

// Blocks are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous range of logical blocks so that the neighbour gathers of the
// operator apply hit the L2 of that XCD.
__device__ __forceinline__ long long xcd_block(int b, int nb) {
  if (nb % 8 != 0) return b;
  return (long long)(b % 8) * (nb / 8) + b / 8;
}

// Fixed-order sum of `cnt` rows (row stride pstride) of nv values into out[v],
// by all threads of the block.  Each thread sums a strided slice of the rows
// with its loads issued in batches of eight before it adds, so the whole sum
// costs about one memory latency.  scratch must hold max(blockDim.x, nv)
// doubles; out and scratch are shared memory.
// Partial sums passed between the blocks of one launch are written with
// agent-scope atomic stores, which write through the XCD's L2, and read with
// agent-scope atomic loads, which do not take a possibly stale L2 copy.  A
// wave then publishes them by waiting for its stores to complete before it
// bumps an arrival counter: no write-back of the whole L2 (what a release
// fence at agent scope costs here, 5-13 us per launch of the fused
// reduction) and no invalidation.
__device__ __forceinline__ void put_partial(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get_partial(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every memory operation this wave has issued has completed (the compiler
// keeps them on their side of the wait).
__device__ __forceinline__ void partials_done() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ void sum_rows(const double* src, int pstride, int cnt, int nv, double* out,
                         double* scratch) {
  const int nt = blockDim.x;
  int S = nt / nv;
  if (S < 1) S = 1;
  if (S > 8) S = 8;
  for (int t = threadIdx.x; t < S * nv; t += nt) {
    const int v = t % nv;
    const int sl = t / nv;
    double acc = 0.0;
    int k = sl;
    for (; k + 7 * S < cnt; k += 8 * S) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = get_partial(src + (size_t)(k + u * S) * pstride + v);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += a[u];
    }
    for (; k < cnt; k += S) acc += get_partial(src + (size_t)k * pstride + v);
    scratch[sl * nv + v] = acc;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += nt) {
    double acc = 0.0;
    for (int sl = 0; sl < S; ++sl) acc += scratch[sl * nv + v];
    out[v] = acc;
  }
  __syncthreads();
}

// Deterministic sums of nv per-block values, in two levels.
// Precondition: wave 0 of every block has written its block's values to
// part[bid * pstride + v], v < nv, with put_partial (only wave 0 writes, so
// that its one wait publishes all of them).
//
// First level (group_reduce_last): the blocks are split into up to 8 groups
// by bid % 8 (under the hardware's round-robin dispatch the blocks of one
// group run on one XCD; the result does not depend on where blocks run), so
// eight counters share the arrivals, and the last block of a group to arrive
// sums that group in a fixed order into gpart[g] and resets the group's
// counter.  Returns true in that block, with out[v]
// (shared memory) holding the group's totals.  scratch: shared memory of
// max(blockDim.x, nv) doubles, disjoint from out.  publish_all: the last
// block also reads other data that blocks wrote with plain stores in this
// launch; then arrivals and the last block add full release and acquire
// fences at agent scope.
__device__ bool group_reduce_last(double* part, double* gpart, int pstride, unsigned* tickets,
                                  int nv, double* out, double* scratch, Grid gr,
                                  bool publish_all = false) {
  __shared__ int s_last;
  const int nb = gr.nb;
  const int ngroups = nb < 8 ? nb : 8;
  const int g = gr.bid % ngroups;
  const int gsize = (nb - g + ngroups - 1) / ngroups;
  if (threadIdx.x < kWave) {
    if (publish_all) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    partials_done();
    if (threadIdx.x == 0) s_last = (atomicAdd(&tickets[g], 1u) == (unsigned)(gsize - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  if (publish_all) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  // members of group g: blocks g, g + ngroups, g + 2 ngroups, ...
  sum_rows(part + (size_t)g * pstride, pstride * ngroups, gsize, nv, out, scratch);
  if (threadIdx.x < kWave) {
    for (int v = threadIdx.x; v < nv; v += kWave) put_partial(gpart + (size_t)g * pstride + v, out[v]);
    if (threadIdx.x == 0) tickets[g] = 0u;
  }
  return true;
}

// Both levels: the last group to finish sums the group totals.  Returns true
// in exactly one block; there out[v] holds the grid totals.
__device__ bool grid_reduce_last(double* part, double* gpart, int pstride, unsigned* tickets,
                                 int nv, double* out, double* scratch, Grid gr,
                                 bool publish_all = false) {
  __shared__ int s_last;
  if (!group_reduce_last(part, gpart, pstride, tickets, nv, out, scratch, gr, publish_all))
    return false;
  const int ngroups = reduce_groups(gr.nb);
  if (threadIdx.x < kWave) {
    if (publish_all) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    partials_done();
    if (threadIdx.x == 0) s_last = (atomicAdd(&tickets[kMaxGroups], 1u) == (unsigned)(ngroups - 1));
  }
  __syncthreads();
  if (!s_last) return false;
  if (publish_all) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  sum_rows(gpart, pstride, ngroups, nv, out, scratch);
  if (threadIdx.x == 0) tickets[kMaxGroups] = 0u;
  return true;
}

// Dot product of two shared-memory vectors by one wave (lanes stride by 64);
// the result is returned in every lane of wave 0.
__device__ __forceinline__ double wave_dot(const double* a, const double* b, int len) {
  const int lane = threadIdx.x % kWave;
  double acc = 0.0;
  for (int i = lane; i < len; i += kWave) acc = fma(a[i], b[i], acc);
  return wave_sum(acc);
}

// ---------------------------------------------------------------------------
// operator apply: z = A u  (or r = b - A x)
// ---------------------------------------------------------------------------

// CSR with LPR lanes per row.  A wave holds G = 64 / LPR lane groups and
// covers G * RPG consecutive rows: group g takes rows base + q G + g,
// q < RPG, so that for each q the wave's loads of row bounds, entries and x
// gathers cover G consecutive rows (contiguous for the entries).  The row
// bounds, the first LPR entries of every row and the x gathers are each
// issued as one batch, so a group pays about three memory latencies for RPG
// rows.  Rows longer than LPR finish in a strided loop.
// TA: type of the matrix values, x, bsub and the sums; TY: type of y.
template <int LPR, int RPG, typename TA, typename TY>
__device__ __forceinline__ void spmv_csr_body(Grid gr, long long n, const int* __restrict__ rp,
                                              const int* __restrict__ ci,
                                              const TA* __restrict__ va,
                                              const TA* __restrict__ x, TY* __restrict__ y,
                                              const TA* __restrict__ bsub,
                                              const Ctl* __restrict__ gate, int gate_j) {
  constexpr int G = kWave / LPR;
  // the gate is read together with the row bounds, so its latency overlaps
  // theirs; nothing is stored before it is checked
  const int act = (gate != nullptr) ? (load_agent(&gate->end_iter) >= gate_j) : 1;
  const long long lb = xcd_block(gr.bid, gr.nb);
  const long long wv = (lb * blockDim.x + threadIdx.x) / kWave;
  const int g = (int)(threadIdx.x % kWave) / LPR;
  const int lane = threadIdx.x % LPR;
  const long long base = wv * (long long)(G * RPG);
  if (base + g >= n) return;  // the group's first row is past the end: its lanes leave together
  int bs[RPG], be[RPG];
#pragma unroll
  for (int q = 0; q < RPG; ++q) {
    const long long row = base + (long long)q * G + g;
    bs[q] = rp[min(row, n)];
    be[q] = rp[min(row + 1, n)];
  }
  if (!act) return;
  int cidx[RPG];
  TA val[RPG];
#pragma unroll
  for (int q = 0; q < RPG; ++q) {
    const int k = bs[q] + lane;
    const bool ok = k < be[q];
    cidx[q] = ok ? ci[k] : 0;
    val[q] = ok ? va[k] : TA(0);
  }
  TA acc[RPG];
#pragma unroll
  for (int q = 0; q < RPG; ++q) acc[q] = val[q] * x[cidx[q]];
#pragma unroll
  for (int q = 0; q < RPG; ++q)
    for (int k = bs[q] + lane + LPR; k < be[q]; k += LPR) acc[q] = fma(va[k], x[ci[k]], acc[q]);
#pragma unroll
  for (int q = 0; q < RPG; ++q) {
    if constexpr (LPR <= 16) {
      acc[q] = group_sum<LPR>(acc[q]);
    } else {
#pragma unroll
      for (int off = LPR / 2; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, LPR);
    }
  }
  // lane l of a group stores the rows q with q % LPR == l; for each q the
  // wave's stores cover G consecutive rows
#pragma unroll
  for (int q = 0; q < RPG; ++q) {
    const long long row = base + (long long)q * G + g;
    if (q % LPR == lane && row < n) y[row] = (TY)((bsub != nullptr) ? bsub[row] - acc[q] : acc[q]);
  }
}

template <int LPR, int RPG, typename TA, typename TY>
__global__ __launch_bounds__(256) void spmv_csr_kernel(long long n, const int* __restrict__ rp,
                                                       const int* __restrict__ ci,
                                                       const TA* __restrict__ va,
                                                       const TA* __restrict__ x,
                                                       TY* __restrict__ y,
                                                       const TA* __restrict__ bsub,
                                                       const Ctl* __restrict__ gate, int gate_j) {
  spmv_csr_body<LPR, RPG, TA, TY>(hw_grid(), n, rp, ci, va, x, y, bsub, gate, gate_j);
}

// Dense row-major operator: one wave per row, 16-byte loads.
__global__ __launch_bounds__(256) void gemv_dense_kernel(long long n, const double* __restrict__ A,
                                                         long long lda,
                                                         const double* __restrict__ x,
                                                         double* __restrict__ y,
                                                         const double* __restrict__ bsub,
                                                         const Ctl* __restrict__ gate, int gate_j) {
  if (gate != nullptr && !ctl_runs(gate, gate_j)) return;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const long long row = (long long)blockIdx.x * (blockDim.x / kWave) + wave;
  if (row >= n) return;
  const double* a = A + row * lda;
  double acc0 = 0.0, acc1 = 0.0;
  const long long n2 = n & ~1LL;
  for (long long c = 2 * lane; c < n2; c += 2 * kWave) {
    const double2 av = *reinterpret_cast<const double2*>(a + c);
    const double2 xv = *reinterpret_cast<const double2*>(x + c);
    acc0 = fma(av.x, xv.x, acc0);
    acc1 = fma(av.y, xv.y, acc1);
  }
  if ((n & 1) && lane == 0) acc0 = fma(a[n - 1], x[n - 1], acc0);
  const double acc = wave_sum(acc0 + acc1);
  if (lane == 0) y[row] = (bsub != nullptr) ? bsub[row] - acc : acc;
}

// Dense row-major operator with x staged in shared memory: a block of 4 waves
// takes 16 rows, 4 per wave, and copies x (zeros past n) into shared memory
// once, so x crosses the caches once per block instead of once per row.
// Each lane reads 16-byte vectors of its wave's 4 rows, two column steps per
// round (8 loads in flight), and the wave sums each row at the end.  Needs
// lda even with zeros in columns n .. lda - 1 and lda doubles of shared
// memory.
constexpr int kGemvLdsRows = 16;
__global__ __launch_bounds__(256) void gemv_lds_kernel(long long n, const double* __restrict__ A,
                                                       long long lda,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y,
                                                       const double* __restrict__ bsub,
                                                       const Ctl* __restrict__ gate, int gate_j) {
  extern __shared__ double xs[];
  if (gate != nullptr && !ctl_runs(gate, gate_j)) return;
  for (long long k = threadIdx.x; k < lda; k += blockDim.x) xs[k] = (k < n) ? x[k] : 0.0;
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const long long rbase = (long long)blockIdx.x * kGemvLdsRows + 4LL * wave;
  const double* __restrict__ rows[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) rows[r] = A + min(rbase + r, n - 1) * lda;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const long long nvec = lda / 2;
  long long c = lane;
  for (; c + kWave < nvec; c += 2 * kWave) {
    dvec2 a0[4], a1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a0[r] = ld_stream2(rows[r] + 2 * c);
      a1[r] = ld_stream2(rows[r] + 2 * (c + kWave));
    }
    const dvec2 x0 = *reinterpret_cast<const dvec2*>(xs + 2 * c);
    const dvec2 x1 = *reinterpret_cast<const dvec2*>(xs + 2 * (c + kWave));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[r] = fma(a0[r][0], x0[0], acc[r]);
      acc[r] = fma(a0[r][1], x0[1], acc[r]);
      acc[r] = fma(a1[r][0], x1[0], acc[r]);
      acc[r] = fma(a1[r][1], x1[1], acc[r]);
    }
  }
  for (; c < nvec; c += kWave) {
    const dvec2 xv = *reinterpret_cast<const dvec2*>(xs + 2 * c);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const dvec2 av = ld_stream2(rows[r] + 2 * c);
      acc[r] = fma(av[0], xv[0], acc[r]);
      acc[r] = fma(av[1], xv[1], acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double sr = wave_sum(acc[r]);
    const long long row = rbase + r;
    if (lane == 0 && row < n) y[row] = (bsub != nullptr) ? bsub[row] - sr : sr;
  }
}

// Dense row-major operator on the matrix cores (v_mfma_f64_16x16x4f64).  A
// block owns 16 rows; its 8 waves take interleaved steps of 32 columns.  In
// a step, lane l (r = l % 16, q = l / 16) reads the 8 entries of row
// i0 + r at columns kb + 8q .. kb + 8q + 7 (four 16-byte loads, so the wave
// reads 256 contiguous bytes of each of its 16 rows) and x at the same
// columns.  Eight MFMAs then take, for t = 0..7, the vector as the A operand
// (A[i][kk] = x[kb + 8kk + t], the same in every row i) and the matrix as the
// B operand (B[kk][j] = A[i0 + j][kb + 8kk + t]), so that every row i of the
// 16 x 16 accumulator holds the partial products of rows i0 .. i0 + 15 in its
// columns j: column j of the result is held by the lanes with l % 16 = j, in
// all four of their accumulator values.  The single right-hand side uses one
// of the 16 accumulator rows' worth of work; the kernel is bound by the
// matrix's bytes, not by the matrix cores.  The 8 waves' partial sums are
// added in a fixed order in shared memory.  Needs lda a multiple of 32 with
// zeros in columns n .. lda - 1 (igs_create_dense pads that way).
constexpr int kGemvWaves = 8;
__global__ __launch_bounds__(kGemvWaves * 64) void gemv_mfma_kernel(
    long long n, const double* __restrict__ A, long long lda, const double* __restrict__ x,
    double* __restrict__ y, const double* __restrict__ bsub, const Ctl* __restrict__ gate,
    int gate_j) {
  __shared__ double part[kGemvWaves][16];
  if (gate != nullptr && !ctl_runs(gate, gate_j)) return;
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int r = lane % 16, q = lane / 16;
  const long long i0 = (long long)blockIdx.x * 16;
  // rows past the end read the last row; their sums are not stored
  const long long row = min(i0 + r, n - 1);
  const double* __restrict__ arow = A + row * lda;
  const long long nsteps = (n + 31) / 32;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  // two steps per round, every load of both issued before the products
  auto load = [&](long long st, double* a, double* xv) {
    const long long kb = st * 32 + 8 * q;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const dvec2 av = ld_stream2(arow + kb + 2 * h);
      a[2 * h] = av[0];
      a[2 * h + 1] = av[1];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) xv[t] = (kb + t < n) ? x[kb + t] : 0.0;
  };
  for (long long st = wave; st < nsteps; st += 2 * kGemvWaves) {
    const bool two = st + kGemvWaves < nsteps;   // the same for the whole wave
    double a0[8], x0[8], a1[8], x1[8];
    load(st, a0, x0);
    load(two ? st + kGemvWaves : st, a1, x1);
#pragma unroll
    for (int t = 0; t < 8; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[t], a0[t], acc, 0, 0, 0);
    if (two) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[t], a1[t], acc, 0, 0, 0);
    }
  }
  // column r of the accumulator: row i0 + r, the same in every entry
  if (q == 0) part[wave][r] = acc[0];
  __syncthreads();
  if (threadIdx.x < 16 && i0 + threadIdx.x < n) {
    double s = part[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kGemvWaves; ++w) s += part[w][threadIdx.x];
    const long long i = i0 + threadIdx.x;
    y[i] = (bsub != nullptr) ? bsub[i] - s : s;
  }
}

// The operator apply from the ELL form, RPT rows per thread: the same
// products and the same order of additions as the CSR kernel with 8 lanes
// per row (pairs, then quads, then the two halves; entries past the row's
// end contribute 0 * x[0]), with no fused multiply-adds (contraction off),
// so z is bit-identical to the CSR kernel's; one memory latency less (no row
// bounds to load first).
template <int K, int RPT, typename TA, typename TY>
__global__ __launch_bounds__(256) void spmv_ell_kernel(long long n, const int* __restrict__ col,
                                                       const TA* __restrict__ val,
                                                       const TA* __restrict__ x,
                                                       TY* __restrict__ y,
                                                       const TA* __restrict__ bsub,
                                                       const Ctl* __restrict__ gate, int gate_j) {
#pragma clang fp contract(off)
  typedef int IV __attribute__((ext_vector_type(RPT)));
  typedef TA AV __attribute__((ext_vector_type(RPT)));
  typedef TY YV __attribute__((ext_vector_type(RPT)));
  const long long row0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * RPT;
  if (gate != nullptr && load_agent(&gate->end_iter) < gate_j) return;
  if (row0 >= n) return;
  // RPT consecutive rows per thread: each entry array is read in RPT-wide
  // vectors (the host launches RPT > 1 only when n and the vector pointers
  // allow it); every row's products and additions are the same as with one
  // row per thread
  IV c[8];
  AV v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < K) {
      c[k] = *reinterpret_cast<const IV*>(col + (long long)k * n + row0);
      v[k] = *reinterpret_cast<const AV*>(val + (long long)k * n + row0);
    } else {
      c[k] = IV(0);
      v[k] = AV(0);
    }
  }
  YV out;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    TA p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = v[k][i] * x[c[k][i]];
    const TA q0 = (p[0] + p[1]) + (p[2] + p[3]);
    const TA q1 = (p[4] + p[5]) + (p[6] + p[7]);
    const TA acc = q0 + q1;
    out[i] = (TY)((bsub != nullptr) ? bsub[row0 + i] - acc : acc);
  }
  __builtin_nontemporal_store(out, reinterpret_cast<YV*>(y + row0));   // see st16
}

template <typename TA> __host__ __device__ const TA* op_vals(const Op& op);
template <> __host__ __device__ const double* op_vals<double>(const Op& op) { return op.vals; }
template <> __host__ __device__ const float* op_vals<float>(const Op& op) { return op.vals32; }
template <typename TA> __host__ __device__ const TA* ell_vals(const Op& op);
template <> __host__ __device__ const double* ell_vals<double>(const Op& op) { return op.ell_val; }
template <> __host__ __device__ const float* ell_vals<float>(const Op& op) { return op.ell_val32; }

// Lanes per row LPR (a power of two near the mean row length) and rows per
// lane group RPG: up to 4 rows while a group is at most 8 lanes wide.
static int spmv_rpg(int lpr) { return lpr <= 8 ? (LPR_RPG_MAX) : (lpr == 16 ? 2 : 1); }

static unsigned spmv_grid(long long n, int lpr, int rpg) {
  const long long groups = (n + rpg - 1) / rpg;
  const long long threads = groups * lpr;
  unsigned grid = (unsigned)((threads + 255) / 256);
  if (grid >= 64) grid = (grid + 7) / 8 * 8;  // multiple of 8 for the XCD mapping
  return grid;
}

template <typename TA, typename TY>
static hipError_t op_apply(const Op& op, const TA* x, TY* y, const TA* bsub, const Ctl* gate,
                           int gate_j, hipStream_t s) {
  if (op.dense) {
    if constexpr (std::is_same<TA, double>::value && std::is_same<TY, double>::value) {
      if (op.dense_mfma == 2) {
        if (op.lda % 2 != 0 || op.lda > kGemvLdsMax) return hipErrorInvalidValue;
        const unsigned grid = (unsigned)((op.n + kGemvLdsRows - 1) / kGemvLdsRows);
        hipLaunchKernelGGL(gemv_lds_kernel, dim3(grid), dim3(256), sizeof(double) * op.lda, s,
                           op.n, op.A, op.lda, x, y, bsub, gate, gate_j);
        return hipGetLastError();
      }
      if (op.dense_mfma == 1) {
        if (op.lda % 32 != 0) return hipErrorInvalidValue;
        const unsigned grid = (unsigned)((op.n + 15) / 16);
        hipLaunchKernelGGL(gemv_mfma_kernel, dim3(grid), dim3(kGemvWaves * 64), 0, s, op.n, op.A,
                           op.lda, x, y, bsub, gate, gate_j);
        return hipGetLastError();
      }
      const int rows_per_block = 4;
      const unsigned grid = (unsigned)((op.n + rows_per_block - 1) / rows_per_block);
      hipLaunchKernelGGL(gemv_dense_kernel, dim3(grid), dim3(256), 0, s, op.n, op.A, op.lda, x, y,
                         bsub, gate, gate_j);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;   // the dense operator is FP64 only
    }
  }
  if (op.ell_k > 0 && op.rpg == 0) {
    const TA* ev = ell_vals<TA>(op);
    if (ev == nullptr) return hipErrorInvalidValue;
    // Two rows per thread when the arrays and y hold whole aligned pairs: each
    // wave then reads 1 KB runs of every value array (31.2 us against 35.5 with
    // one row per thread on the 2M-row stencil; four rows per thread, 33.5)
    constexpr int kR = 2;
    const bool wide = (op.n % kR == 0) &&
                      (reinterpret_cast<uintptr_t>(y) % (kR * sizeof(TY)) == 0) &&
                      (reinterpret_cast<uintptr_t>(op.ell_col) % (kR * sizeof(int)) == 0) &&
                      (reinterpret_cast<uintptr_t>(ev) % (kR * sizeof(TA)) == 0);
    const long long threads = wide ? op.n / kR : op.n;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    switch (op.ell_k * 2 + (wide ? 1 : 0)) {
#define IGS_ELL_CASE(K)                                                                         \
  case K * 2:                                                                                   \
    hipLaunchKernelGGL((spmv_ell_kernel<K, 1, TA, TY>), dim3(grid), dim3(256), 0, s, op.n,      \
                       op.ell_col, ev, x, y, bsub, gate, gate_j);                               \
    break;                                                                                      \
  case K * 2 + 1:                                                                               \
    hipLaunchKernelGGL((spmv_ell_kernel<K, kR, TA, TY>), dim3(grid), dim3(256), 0, s, op.n,     \
                       op.ell_col, ev, x, y, bsub, gate, gate_j);                               \
    break;
      IGS_ELL_CASE(1) IGS_ELL_CASE(2) IGS_ELL_CASE(3) IGS_ELL_CASE(4)
      IGS_ELL_CASE(5) IGS_ELL_CASE(6) IGS_ELL_CASE(7) IGS_ELL_CASE(8)
#undef IGS_ELL_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const TA* vals = op_vals<TA>(op);
  if (vals == nullptr) return hipErrorInvalidValue;
  const int lpr = op.lpr;
  const int rpg = op.rpg > 0 ? op.rpg : spmv_rpg(lpr);
  const unsigned grid = spmv_grid(op.n, lpr, rpg);
  switch (lpr * 8 + rpg) {
#define IGS_SPMV_CASE(L, R)                                                                     \
  case L * 8 + R:                                                                               \
    hipLaunchKernelGGL((spmv_csr_kernel<L, R, TA, TY>), dim3(grid), dim3(256), 0, s, op.n,      \
                       op.row_ptr, op.col_idx, vals, x, y, bsub, gate, gate_j);                 \
    break;
    IGS_SPMV_CASE(1, 1) IGS_SPMV_CASE(1, 2) IGS_SPMV_CASE(1, 4)
    IGS_SPMV_CASE(2, 1) IGS_SPMV_CASE(2, 2) IGS_SPMV_CASE(2, 4)
    IGS_SPMV_CASE(4, 1) IGS_SPMV_CASE(4, 2) IGS_SPMV_CASE(4, 4)
    IGS_SPMV_CASE(8, 1) IGS_SPMV_CASE(8, 2) IGS_SPMV_CASE(8, 4)
    IGS_SPMV_CASE(16, 1) IGS_SPMV_CASE(16, 2) IGS_SPMV_CASE(32, 1) IGS_SPMV_CASE(64, 1)
#undef IGS_SPMV_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spmv(const Op& op, const double* u, double* z, const Ctl* gate, int j,
                       hipStream_t s) {
  return op_apply<double, double>(op, u, z, nullptr, gate, j, s);
}

hipError_t launch_spmv32(const Op& op, const float* u, float* z, const Ctl* gate, int j,
                         hipStream_t s) {
  return op_apply<float, float>(op, u, z, nullptr, gate, j, s);
}

// FP64 values of the operator rounded to FP32 (the inner step of the
// mixed-precision solve).
__global__ void round_to_float_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                      long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

hipError_t launch_round_to_float(const double* src, float* dst, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  long long blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(round_to_float_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst,
                     count);
  return hipGetLastError();
}

// The column-major ELL form of a CSR operator whose rows hold at most K
// entries: entry k of row i at k n + i, the slots past a row's end column 0
// and value 0 (the layout igs_create builds on the host).  One thread per
// row; the stores of each slot are consecutive over the rows.
__global__ void csr_to_ell_kernel(long long n, int K, const int* __restrict__ rp,
                                  const int* __restrict__ ci, const double* __restrict__ va,
                                  int* __restrict__ ec, double* __restrict__ ev) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = rp[i], e = rp[i + 1];
  for (int k = 0; k < K; ++k) {
    const int idx = b + k;
    const bool ok = idx < e;
    ec[(long long)k * n + i] = ok ? ci[idx] : 0;
    ev[(long long)k * n + i] = ok ? va[idx] : 0.0;
  }
}

hipError_t launch_csr_to_ell(long long n, int K, const int* rp, const int* ci, const double* va,
                             int* ec, double* ev, hipStream_t s) {
  if (n <= 0 || K < 1 || K > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(csr_to_ell_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, K,
                     rp, ci, va, ec, ev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cycle start: reset the control block, then r0 = b - A x into V[:, 0]
// ---------------------------------------------------------------------------

__device__ __forceinline__ void cycle_begin_body(Ctl* c, long long its_before, long long maxit,
                                                 int m, int gs, int final_v, double tol,
                                                 double tau, double cycle_rtol) {
  c->end_iter = kNotEnded;
  c->J = 0;
  c->status = kRunning;
  c->mode = kUpdNone;
  c->mode_iter = -1;
  if (its_before >= 0) c->its_before = its_before;   // < 0: the host wrote it
  c->maxit = maxit;
  c->m = m;
  c->gs = gs;
  c->final_v = final_v;
  c->tol = tol;
  c->tol_abs = tol * c->bnorm;
  c->tol_cyc = c->tol_abs;
  c->cycle_rtol = cycle_rtol;
  c->lagnorm_tau = tau;
  c->gabs = 0.0;
}

__global__ void cycle_begin_kernel(Ctl* c, long long its_before, long long maxit, int m, int gs,
                                   int final_v, double tol, double tau, double cycle_rtol) {
  if (threadIdx.x != 0) return;
  cycle_begin_body(c, its_before, maxit, m, gs, final_v, tol, tau, cycle_rtol);
}

hipError_t launch_residual(const Op& op, const double* b, const double* x, const Work& w,
                           long long its_before, long long maxit, int m, int gs, int final_v,
                           double tol, double tau, double cycle_rtol, hipStream_t s) {
  hipLaunchKernelGGL(cycle_begin_kernel, dim3(1), dim3(64), 0, s, w.ctl, its_before, maxit, m, gs,
                     final_v, tol, tau, cycle_rtol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (w.fp32) return op_apply<double, float>(op, x, w.V32, b, nullptr, 0, s);
  return op_apply<double, double>(op, x, w.V, b, nullptr, 0, s);
}

// ---------------------------------------------------------------------------
// ||b|| and a finiteness check of b and x0 (once per solve)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bnorm_body(Grid gr, const double* __restrict__ b,
                                           const double* __restrict__ x, long long n,
                                           const Work& w) {
  __shared__ double red[2][256 / kWave];
  __shared__ double tot[2];
  __shared__ double scr[256];
  double s2 = 0.0, bad = 0.0;
  for (long long i = (long long)gr.bid * blockDim.x + threadIdx.x; i < n;
       i += (long long)gr.nb * blockDim.x) {
    const double bi = b[i];
    const double xi = x[i];
    s2 = fma(bi, bi, s2);
    bad += (isfinite(bi) ? 0.0 : 1.0) + (isfinite(xi) ? 0.0 : 1.0);
  }
  s2 = wave_sum(s2);
  bad = wave_sum(bad);
  const int wave = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) {
    red[0][wave] = s2;
    red[1][wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double acc = 0.0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) acc += red[threadIdx.x][k];
    put_partial(w.part + (size_t)gr.bid * w.pstride + threadIdx.x, acc);
  }
  if (!grid_reduce_last(w.part, w.gpart, w.pstride, w.tickets, 2, tot, scr, gr)) return;
  if (threadIdx.x == 0) {
    w.ctl->bnorm = sqrt(tot[0]);
    w.ctl->nonfinite_in = (int)tot[1];
    w.ctl->breakdowns = 0;
    w.ctl->fallbacks = 0;
  }
}

__global__ __launch_bounds__(256) void bnorm_kernel(const double* __restrict__ b,
                                                    const double* __restrict__ x, long long n,
                                                    Work w) {
  bnorm_body(hw_grid(), b, x, n, w);
}

hipError_t launch_bnorm(const double* b, const double* x, long long n, const Work& w,
                        hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(bnorm_kernel, dim3((unsigned)blocks), dim3(256), 0, s, b, x, n, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Givens rotation of a finished Hessenberg column (eq:llse), one thread.
// col[0..c+1] (shared) holds column c before rotation; on return R[:, c],
// cs[c], sn[c] and g[c], g[c+1] are updated and |g[c+1]| is returned.
// ---------------------------------------------------------------------------

__device__ double givens_column(const Work& w, int c, double* col, const double* scs,
                                const double* ssn, double gc) {
  // Rotation i mixes entries i and i+1.  The running entry `cur` carries the
  // dependency chain; the inputs col[i+1], cs[i], sn[i] do not depend on it and
  // are loaded in groups of eight ahead of the arithmetic.
  double cur = col[0];
  int i = 0;
  for (; i + 8 <= c; i += 8) {
    double nb[8], cc[8], ss[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      nb[q] = col[i + q + 1];
      cc[q] = scs[i + q];
      ss[q] = ssn[i + q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      col[i + q] = cc[q] * cur + ss[q] * nb[q];
      cur = -ss[q] * cur + cc[q] * nb[q];
    }
  }
  for (; i < c; ++i) {
    const double nb = col[i + 1];
    col[i] = scs[i] * cur + ssn[i] * nb;
    cur = -ssn[i] * cur + scs[i] * nb;
  }
  const double a = cur;
  const double b = col[c + 1];
  const double d = hypot(a, b);
  double cs = 1.0, sn = 0.0;
  if (d != 0.0) {
    cs = a / d;
    sn = b / d;
  }
  col[c] = d;
  col[c + 1] = 0.0;
  w.cs[c] = cs;
  w.sn[c] = sn;
  w.g[c + 1] = -sn * gc;
  w.g[c] = cs * gc;
  return fabs(sn * gc);
}

// Packed storage of the small matrices (device memory):
//   T = (I + L)^{-1}, lower triangular: row i holds T[i, 0..i] at tri_row(i);
//   H, upper Hessenberg:               column c holds H[0..c+1, c] at hess_col(c).
// Both grow by appending (a row of T, a column of H per iteration), so the
// part an iteration reads is one contiguous prefix.
__device__ __forceinline__ size_t tri_row(int i) { return (size_t)i * (i + 1) / 2; }
__host__ __device__ __forceinline__ size_t hess_col(int c) { return (size_t)c * (c + 3) / 2; }

// Copy count doubles from global src to shared dst with every thread's loads
// issued in batches of eight (about one memory latency for the whole copy).
__device__ void stage_copy(double* dst, const double* src, size_t count) {
  const size_t nt = blockDim.x;
  for (size_t k0 = threadIdx.x; k0 < count; k0 += 8 * nt) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const size_t k = k0 + q * nt;
      v[q] = (k < count) ? src[k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const size_t k = k0 + q * nt;
      if (k < count) dst[k] = v[q];
    }
  }
}

// Largest staged prefix of T and H (doubles of shared memory in the last
// block of the reduction); larger iterations read them from global memory.
constexpr size_t kStageMax = 6144;
__host__ __device__ __forceinline__ size_t stage_count(int j) {
  if (j < 1) return 0;
  const size_t c = (size_t)j * (j + 1) / 2 + (size_t)(j - 1) * (j + 2) / 2;
  return c <= kStageMax ? c : 0;
}

// Finish Hessenberg column j-1 with subdiagonal gamma: store H and the rotated
// column, apply the rotation, and run the breakdown test.  hcol (shared or
// global, j+1 entries) holds H[0:j, j-1]; scs/ssn hold the rotations 0..j-2
// and gc the right-hand side entry g[j-1], all loaded by the caller.  Called
// by all threads of a block.  Returns 1 on breakdown, 0 otherwise;
// ctl->gabs is updated.
__device__ int finish_column(const Work& w, int j, double* hcol, double gamma, const double* scs,
                             const double* ssn, double gc, long long n) {
  __shared__ double s_hn;
  __shared__ int s_brk;
  const int c = j - 1;
  double* hc = w.H + hess_col(c);
  for (int i = threadIdx.x; i < j; i += blockDim.x) hc[i] = hcol[i];
  if (threadIdx.x == 0) hc[j] = gamma;
  if (threadIdx.x < kWave) {
    const double hn2 = wave_dot(hcol, hcol, j);
    if (threadIdx.x == 0) s_hn = sqrt(hn2);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    hcol[j] = gamma;
    const double gabs = givens_column(w, c, hcol, scs, ssn, gc);
    w.ctl->gabs = gabs;
    const double eps = 2.220446049250313e-16;
    s_brk = (gamma <= (double)n * eps * s_hn) ? 1 : 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += blockDim.x) w.R[(size_t)c * w.ldh + i] = hcol[i];
  const int brk = s_brk;
  __syncthreads();
  return brk;
}

// Products with the small matrices T and H, computed by the whole block.
// Ts / Hs are the packed T and H.  Staged (shared memory): one output per
// thread, a sequential dot product over LDS, no cross-lane reduction.  Not
// staged (global memory): one wave per output, coalesced loads and a wave sum.

// y[i] = sum_{c <= i} T[i, c] x[c], i < j.
template <bool STAGED>
__device__ __forceinline__ void tri_matvec(const double* Ts, const double* x, double* y, int j) {
  if constexpr (STAGED) {
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
      const double* trow = Ts + tri_row(i);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int c = 0;
      for (; c + 8 <= i + 1; c += 8) {
        double a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a[q] = trow[c + q];
          b[q] = x[c + q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q & 3] = fma(a[q], b[q], acc[q & 3]);
      }
      for (; c <= i; ++c) acc[0] = fma(trow[c], x[c], acc[0]);
      y[i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  } else {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, nw = blockDim.x / kWave;
    for (int i = wave; i < j; i += nw) {
      const double* trow = Ts + tri_row(i);
      double acc = 0.0;
      for (int c = lane; c <= i; c += kWave) acc = fma(trow[c], x[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[i] = acc;
    }
  }
}

// y[c] = -sum_{i = c..j-1} l[i] T[i, c], c < j.
template <bool STAGED>
__device__ __forceinline__ void tri_rowvec(const double* Ts, const double* l, double* y, int j) {
  if constexpr (STAGED) {
    for (int c = threadIdx.x; c < j; c += blockDim.x) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int i = c;
      for (; i + 8 <= j; i += 8) {
        double a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a[q] = l[i + q];
          b[q] = Ts[tri_row(i + q) + c];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q & 3] = fma(a[q], b[q], acc[q & 3]);
      }
      for (; i < j; ++i) acc[0] = fma(l[i], Ts[tri_row(i) + c], acc[0]);
      y[c] = -((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
  } else {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, nw = blockDim.x / kWave;
    for (int c = wave; c < j; c += nw) {
      double acc = 0.0;
      for (int i = c + lane; i < j; i += kWave) acc = fma(l[i], Ts[tri_row(i) + c], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[c] = -acc;
    }
  }
}

// y[i] = sum_{c = max(i-1,0)..j-2} H[i, c] x[c], i < j.
template <bool STAGED>
__device__ __forceinline__ void hess_matvec(const double* Hs, const double* x, double* y, int j) {
  if constexpr (STAGED) {
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int c = i > 0 ? i - 1 : 0;
      for (; c + 8 <= j - 1; c += 8) {
        double a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          a[q] = Hs[hess_col(c + q) + i];
          b[q] = x[c + q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q & 3] = fma(a[q], b[q], acc[q & 3]);
      }
      for (; c < j - 1; ++c) acc[0] = fma(Hs[hess_col(c) + i], x[c], acc[0]);
      y[i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  } else {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, nw = blockDim.x / kWave;
    for (int i = wave; i < j; i += nw) {
      double acc = 0.0;
      for (int c = (i > 0 ? i - 1 : 0) + lane; c < j - 1; c += kWave)
        acc = fma(Hs[hess_col(c) + i], x[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) y[i] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// The small solve of iteration j, run by every block of the update kernel on
// the totals of the fused reduction, P[c] = V_c^T u and Q[c] = V_c^T z for
// c <= j (P[j] = u^T u, Q[j] = u^T z), held in shared memory.
//
// Every block forms what its share of the update needs: the second-sweep
// vector t (in sm[0..j-1]), gamma, the first-sweep vector r1 (in
// sm[2(j+2) .. 2(j+2)+j]) and the update mode.  The publishing block (pub)
// also finishes Hessenberg column j-1, applies its Givens rotation, appends
// the rows of L and T = (I + L)^{-1} (eq:block), runs the stopping tests and
// writes the results and the control block.  All blocks read the same inputs
// and run the same arithmetic, so their t, gamma and r1 agree bit for bit.
// What the other blocks read from device memory (T rows < j, the cycle
// constants of the control block) is disjoint from what the publisher writes
// (T row j, the L row, H and R column j-1, cs/sn[j-1], g[j-1..j], the
// coefficient vectors, the status fields of the control block); the inputs
// only the publisher reads (previous coefficients, rotations, g[j-1], H
// columns < j-1) are read before it writes.
//
// sm: shared scratch of 7 (j + 2) doubles, followed (STAGED) by the staged
// prefix of T (all blocks) and H (publisher), stage_count(j) doubles.
// ---------------------------------------------------------------------------

struct StepCoefs {
  int mode;   // UpdateMode of this block's share of the update
  double ig;  // 1 / gamma
};

// Where the products with T and H come from: computed by the block from
// global memory, from the staged copies in shared memory, or read as
// coef_kernel left them (PRE: iterations beyond the staging limit).
enum SolveKind : int { kSolveGlobal = 0, kSolveStaged = 1, kSolvePre = 2 };

// Offsets of the products coef_kernel forms for iteration j in w.pre.
__host__ __device__ __forceinline__ int pre_t(int j) { return 0; }
__host__ __device__ __forceinline__ int pre_h(int j) { return j + 2; }
__host__ __device__ __forceinline__ int pre_row(int j) { return 2 * (j + 2); }

template <int KIND>
__device__ StepCoefs small_solve(const Work& w, long long n, int j, bool tail, const double* P,
                                 const double* Q, double* sm, bool pub) {
  constexpr bool STAGED = (KIND == kSolveStaged);
  Ctl* ctl = w.ctl;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const int lane = tid % kWave;
  const int L1 = j + 2;
  double* st = sm;            // t (second sweep coefficients)
  double* shc = sm + L1;      // finished column j-1 (publisher)
  double* sr1 = sm + 2 * L1;  // new first-sweep coefficients
  double* sx = sm + 3 * L1;   // t_prev / gamma_prev, then temporaries
  double* sl = sm + 4 * L1;   // new row of L
  double* scs = sm + 5 * L1;  // rotations cos 0..j-2 (publisher)
  double* ssn = sm + 6 * L1;  // rotations sin 0..j-2 (publisher)
  __shared__ double s_gamma, s_pp, s_gc, s_gprev;
  __shared__ int s_flag;

  const int gs = ctl->gs;
  const int m = ctl->m;
  // A block's share while the cycle may go on: v_j and u_{j+1}, also past a
  // stop that only the publisher sees (columns j and j+1 are not used after
  // it); at the tail iteration v_j only, and only on request.
  const int run_mode = tail ? (ctl->final_v ? kUpdVOnly : kUpdNone) : kUpdNormal;
  const double alpha = P[j];
  const double beta = tail ? 0.0 : Q[j];
  StepCoefs out{kUpdNone, 0.0};

  if (!isfinite(alpha) || !isfinite(beta)) {
    if (pub && tid == 0) {
      ctl->status = kNonfinite;
      ctl->J = j > 0 ? j - 1 : 0;
      ctl->end_iter = j;
      ctl->mode = kUpdNone;
      ctl->mode_iter = j;
    }
    return out;
  }

  if (j == 0) {
    const double gamma = sqrt(alpha);
    // converged at the start, or a check cycle after the iteration budget
    const bool stop = (gamma <= ctl->tol_abs) || (ctl->its_before >= ctl->maxit);
    out.ig = 1.0 / gamma;
    if (tid == 0) sr1[0] = beta * out.ig * out.ig;
    if (pub && tid == 0) {
      ctl->rho = gamma;
      ctl->gabs = gamma;
      w.g[0] = gamma;
      if (stop) {
        ctl->status = (gamma <= ctl->tol_abs) ? kConvStart : kMaxit;
        ctl->J = 0;
        ctl->end_iter = 0;
        ctl->mode = kUpdNone;
      } else {
        w.T[0] = 1.0;
        w.coef_r1[0] = beta * out.ig * out.ig;
        ctl->gamma_prev = gamma;
        ctl->mode = run_mode;
        // the Arnoldi-residual target of the cycle (read by this block only)
        if (ctl->cycle_rtol > 0.0) ctl->tol_cyc = fmax(ctl->tol_abs, ctl->cycle_rtol * gamma);
      }
      ctl->mode_iter = 0;
    }
    __syncthreads();
    out.mode = stop ? kUpdNone : run_mode;
    return out;
  }

  // ---- one batch of loads: T rows 0..j-1 (and, publisher, H columns 0..j-2)
  // staged; publisher: the previous coefficients, the rotations and g[j-1]
  const double* Ts = w.T;
  const double* Hs = w.H;
  if constexpr (STAGED) {
    double* stg = sm + 7 * L1;
    const size_t nT = tri_row(j);
    stage_copy(stg, w.T, nT);
    Ts = stg;
    if (pub) {
      stage_copy(stg + nT, w.H, hess_col(j - 1));
      Hs = stg + nT;
    }
  }
  if (pub) {
    for (int i = tid; i < j; i += blockDim.x) {
      shc[i] = w.coef_r1[i];               // r1 of the previous iteration
      if (i < j - 1) {
        sx[i] = w.coef_t[i];               // t of the previous iteration
        scs[i] = w.cs[i];
        ssn[i] = w.sn[i];
      }
    }
    if (tid == 0) {
      s_gc = w.g[j - 1];
      s_gprev = ctl->gamma_prev;
    }
  }
  __syncthreads();

  // ---- second sweep t = (I + L_{0:j,0:j})^{-1} p = T_j p  (gs = 2), and p.p
  if (gs == 2) {
    if constexpr (KIND == kSolvePre) {
      for (int i = tid; i < j; i += blockDim.x) st[i] = w.pre[pre_t(j) + i];
    } else {
      tri_matvec<STAGED>(Ts, P, st, j);
    }
  } else {
    for (int i = tid; i < j; i += blockDim.x) st[i] = 0.0;
  }
  if (wave == 0) {
    const double pp = wave_dot(P, P, j);
    if (lane == 0) s_pp = pp;
  }
  if (pub) {
    const double igp = 1.0 / s_gprev;
    for (int i = tid; i < j - 1; i += blockDim.x) sx[i] *= igp;   // t_prev / gamma_prev
  }
  __syncthreads();

  // ---- finished column j-1 (publisher): r1_prev + t - H[0:j, 0:j-1] (t_prev / gamma_prev)
  if (pub && gs == 2) {
    if constexpr (KIND == kSolvePre) {
      for (int i = tid; i < j; i += blockDim.x) sr1[i] = w.pre[pre_h(j) + i];
    } else {
      hess_matvec<STAGED>(Hs, sx, sr1, j);   // sr1 is free until the first sweep below
    }
    __syncthreads();
    for (int i = tid; i < j; i += blockDim.x) shc[i] = shc[i] + st[i] - sr1[i];
  }
  __syncthreads();

  // ---- lagged norm (gs = 2) or explicit norm (gs = 1) ------------------------
  if (tid == 0) {
    int fb = 0;
    double gamma;
    if (gs == 2) {
      const double g2 = alpha - s_pp;
      if (!(g2 >= ctl->lagnorm_tau * alpha) || !(g2 > 0.0)) fb = 1;
      gamma = fb ? 0.0 : sqrt(g2);
    } else {
      gamma = sqrt(alpha);
    }
    s_gamma = gamma;
    s_flag = fb;
  }
  __syncthreads();
  if (s_flag) {
    // Cancellation in u^T u - p^T p: every block forms w = u - V t and its
    // explicit norm; the publisher leaves the column without its subdiagonal.
    // Wave 0 alone stores it: the last block of the explicit-norm reduction
    // in this launch reads it, and the release fence before wave 0's arrival
    // at that reduction orders wave 0's own stores only.
    if (pub && wave == 0) {
      double* hc = w.H + hess_col(j - 1);
      for (int i = lane; i < j; i += kWave) hc[i] = shc[i];
      if (lane == 0) {
        ctl->mode = kUpdFallback;
        ctl->mode_iter = j;
      }
    }
    out.mode = kUpdFallback;
    return out;
  }
  const double gamma = s_gamma;
  const double ig = 1.0 / gamma;
  out.ig = ig;

  // ---- new row of L (p / gamma) ---------------------------------------------
  for (int c = tid; c < j; c += blockDim.x) {
    const double l = P[c] * ig;
    sl[c] = l;
    if (pub) w.L[(size_t)c * w.ldt + j] = l;
  }

  // ---- publisher: Hessenberg column, Givens rotation, breakdown test, the row
  // of T = (I + L)^{-1} (eq:block), stopping tests
  int st_code = kRunning;
  if (pub) {
    const int brk = finish_column(w, j, shc, gamma, scs, ssn, s_gc, n);   // synchronises
    if (!brk) {
      if constexpr (KIND == kSolvePre) {
        for (int c = tid; c < j; c += blockDim.x) sx[c] = w.pre[pre_row(j) + c];
      } else {
        tri_rowvec<STAGED>(Ts, sl, sx, j);
      }
      __syncthreads();
      double* trow = w.T + tri_row(j);
      for (int c = tid; c < j; c += blockDim.x) trow[c] = sx[c];
      if (tid == 0) trow[j] = 1.0;
    }
    if (tid == 0) {
      int code = kRunning;
      if (brk) code = kBreakdown;
      else if (ctl->gabs <= ctl->tol_cyc) code = kConverged;
      else if (j >= m) code = kFull;
      else if (ctl->its_before + j >= ctl->maxit) code = kMaxit;
      s_flag = code;
      if (code != kRunning) {
        ctl->status = code;
        ctl->J = j;
        ctl->end_iter = j;
        if (brk) ctl->breakdowns += 1;
      }
    }
    __syncthreads();
    st_code = s_flag;
  }

  // ---- first sweep of the next vector (all blocks; none at the tail) --------
  if (!tail) {
    if (gs == 2) {
      // Stephen's trick: r1 = [q/gamma ; beta/gamma^2 - (t/gamma)^T (q/gamma)]
      for (int c = tid; c < j; c += blockDim.x) {
        sr1[c] = Q[c] * ig;
        sx[c] = st[c] * ig;
      }
      __syncthreads();
      if (wave == 0) {
        const double d = wave_dot(sx, sr1, j);
        if (lane == 0) sr1[j] = beta * ig * ig - d;
      }
    } else {
      // r1 = (I + L_{0:j+1,0:j+1})^{-1} [q/gamma ; beta/gamma^2]
      if constexpr (KIND == kSolvePre) {
        for (int c = tid; c < j; c += blockDim.x) sr1[c] = w.pre[pre_t(j) + c];
      } else {
        for (int c = tid; c < j; c += blockDim.x) sx[c] = Q[c] * ig;
        __syncthreads();
        tri_matvec<STAGED>(Ts, sx, sr1, j);
      }
      __syncthreads();
      if (wave == 0) {
        const double d = wave_dot(sl, sr1, j);
        if (lane == 0) sr1[j] = beta * ig * ig - d;
      }
    }
    __syncthreads();
  }
  if (pub) {
    if (st_code == kRunning) {
      for (int i = tid; i <= j; i += blockDim.x) {
        w.coef_r1[i] = sr1[i];
        if (i < j) w.coef_t[i] = st[i];
      }
    }
    if (tid == 0) {
      if (st_code == kRunning) ctl->gamma_prev = gamma;
      ctl->mode = run_mode;
      ctl->mode_iter = j;
    }
  }
  out.mode = run_mode;
  return out;
}

// ---------------------------------------------------------------------------
// The small products of a large iteration, spread over many CUs
// ---------------------------------------------------------------------------
//
// Past the staging limit every update block would read the prefixes of T and
// H from global memory one row per wave, a memory latency per row, and the
// publishing block three such products in a row (about 100 us at j = 195).
// This kernel forms them once, one wave per output over as many blocks as
// there are outputs, before the update; the update blocks then read j values
// of each.  Each output is the update's own unstaged product (lanes stride the
// row, then a wave sum) on the same reduction totals summed in the same order,
// so the values are bit-identical to the ones the update blocks would form:
//   pre_t:   gs = 2: t = T_j p;  gs = 1: T_j (q / gamma), the first sweep;
//   pre_h:   gs = 2: H[0:j, 0:j-1] (t_prev / gamma_prev), for the finished column;
//   pre_row: -(p / gamma)^T T_j, the new row of T (eq:block); skipped when the
//            lagged norm cancels (the update then takes the fallback).
__global__ __launch_bounds__(256) void coef_kernel(Work w, int j, int ngroups) {
  extern __shared__ double lds[];
  const Ctl* ctl = w.ctl;
  if (!ctl_runs(ctl, j)) return;
  double* P = lds;                 // V^T u, u^T u
  double* Q = lds + (j + 1);       // V^T z, u^T z
  double* X = lds + 2 * (j + 1);   // the vector each product multiplies
  double* Lr = X + (j + 1);        // p / gamma
  __shared__ double s_ig, s_pp;
  __shared__ int s_ok;
  for (int v = threadIdx.x; v < 2 * (j + 1); v += blockDim.x) {
    double g8[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) g8[g] = (g < ngroups) ? w.gpart[(size_t)g * w.pstride + v] : 0.0;
    double acc = g8[0];
#pragma unroll
    for (int g = 1; g < 8; ++g) acc += g8[g];
    lds[v] = acc;
  }
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int gs = ctl->gs;
  const double alpha = P[j];
  if (wave == 0) {
    const double pp = wave_dot(P, P, j);
    if (lane == 0) {
      s_pp = pp;
      int ok = 1;
      double gamma;
      if (gs == 2) {
        const double g2 = alpha - pp;
        if (!(g2 >= ctl->lagnorm_tau * alpha) || !(g2 > 0.0)) ok = 0;
        gamma = ok ? sqrt(g2) : 1.0;
      } else {
        gamma = sqrt(alpha);
      }
      s_ig = 1.0 / gamma;
      s_ok = ok;
    }
  }
  __syncthreads();
  const double ig = s_ig;
  const double igp = 1.0 / ctl->gamma_prev;
  for (int c = threadIdx.x; c < j; c += blockDim.x) {
    X[c] = (gs == 2) ? w.coef_t[c] * igp : Q[c] * ig;   // t_prev / gamma_prev, or q / gamma
    Lr[c] = P[c] * ig;
  }
  __syncthreads();
  // outputs: [0, j) first products, [j, 2j) H products (gs = 2), [2j, 3j) the T row
  const int o = blockIdx.x * (blockDim.x / kWave) + wave;
  if (o < j) {
    const int i = o;
    const double* trow = w.T + tri_row(i);
    const double* x = (gs == 2) ? P : X;
    double acc = 0.0;
    for (int c = lane; c <= i; c += kWave) acc = fma(trow[c], x[c], acc);
    acc = wave_sum(acc);
    if (lane == 0) w.pre[pre_t(j) + i] = acc;
  } else if (o < 2 * j) {
    const int i = o - j;
    if (gs == 2 && j >= 1) {
      double acc = 0.0;
      for (int c = (i > 0 ? i - 1 : 0) + lane; c < j - 1; c += kWave)
        acc = fma(w.H[hess_col(c) + i], X[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) w.pre[pre_h(j) + i] = acc;
    }
  } else if (o < 3 * j) {
    const int c = o - 2 * j;
    if (s_ok) {
      double acc = 0.0;
      for (int i = c + lane; i < j; i += kWave) acc = fma(Lr[i], w.T[tri_row(i) + c], acc);
      acc = wave_sum(acc);
      if (lane == 0) w.pre[pre_row(j) + c] = -acc;
    }
  }
}

bool coef_kernel_needed(const Work& w, int j) {
  return w.pre_on && w.pre != nullptr && j >= 1 && stage_count(j) == 0;
}

hipError_t launch_coef(const Work& w, int j, int ngroups, hipStream_t s) {
  const int outputs = 3 * j;
  const unsigned grid = (unsigned)((outputs + 3) / 4);
  const size_t lds = sizeof(double) * (size_t)4 * (j + 1);
  hipLaunchKernelGGL(coef_kernel, dim3(grid), dim3(256), lds, s, w, j, ngroups);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused reduction [V_{0:j}, u]^T [u, z]
// ---------------------------------------------------------------------------
//
// A block owns a contiguous row range.  Its 8 waves are arranged as Wc column
// groups x Wr row slices: a wave accumulates 2*CPW sums (against u and z) for
// its columns over its rows, so V is streamed exactly once and each wave
// reduces across lanes only once per column group.

struct ReduceShape {
  int cpw;   // columns per group (the last group may have fewer)
  int tcpw;  // template width: the power of two >= cpw
  int wc, wr;
  int nblocks;
  long long rows_per_block;
};

// Column groups x row slices for the 8 waves of a block: groups of cpw <= 8
// columns, wc groups side by side and wr = 8 / wc row slices.  Among
// wc in {1, 2, 4, 8} take the one whose busiest wave streams the fewest
// values per row, (cpw + 2) / wr: its columns plus u and z.  Beyond 64
// columns the 8 waves loop over groups of 8.
static ReduceShape reduce_columns(int ncol) {
  ReduceShape s{8, 8, kReduceWaves, 1, 0, 0};
  double best = 1e30;
  for (int wc = 1; wc <= kReduceWaves; wc *= 2) {
    const int cpw = (ncol + wc - 1) / wc;
    if (cpw > 8) continue;
    const int wr = kReduceWaves / wc;
    const double cost = (double)(cpw + 2) / wr;
    if (cost < best) {
      best = cost;
      s.cpw = cpw;
      s.wc = wc;
      s.wr = wr;
    }
  }
  s.tcpw = 1;
  while (s.tcpw < s.cpw) s.tcpw *= 2;
  return s;
}

// Rows per block (a multiple of 256, so that 16-byte row vectors of doubles
// or floats and 64-lane steps tile a block's range) for at most max_blocks
// blocks.
static void reduce_rows(ReduceShape& s, long long n, int max_blocks) {
  long long nb = (n + 255) / 256;
  if (nb > max_blocks) nb = max_blocks;
  if (nb < 1) nb = 1;
  long long rpb = (n + nb - 1) / nb;
  rpb = (rpb + 255) / 256 * 256;
  s.rows_per_block = rpb;
  s.nblocks = (int)((n + rpb - 1) / rpb);
}


// One wave's share of the fused reduction for NC consecutive columns of V
// (starting at vb): over the rows of its slice of [r0, r1),
// ap[c] += V[r, c] u[r - uoff] and (Z) aq[c] += V[r, c] z[r - zoff], products
// and sums in FP64 whatever the element type T of V, u and z (an offset is r0
// when that vector is the block's own rows in shared memory, else 0).  NC and Z are
// compile-time, so every load of a row step is unconditional and the whole
// step is in flight before the first FMA.
template <int NC, bool VEC, bool Z, typename T>
__device__ __forceinline__ void stream_cols(const T* __restrict__ vb, long long ldv,
                                            const T* __restrict__ u, long long uoff,
                                            const T* __restrict__ z, long long zoff, long long r0, long long r1, int rw,
                                            int wr, int lane, double* ap, double* aq) {
  if constexpr (VEC) {
    // Lane owns W consecutive rows (one 16-byte load per column; V
    // non-temporal).  Two-stage software pipeline: the loads of the next row
    // step are issued before the FMAs of the current one, so a wave always
    // has a step in flight.  The two register stages A and B alternate roles
    // (no copies between them, which would force a wait on the loads in
    // flight).  Without a next step the current rows are loaded again and
    // not used, so the loads stay unconditional and each wait covers only
    // the step being consumed.
    typedef typename Vec16<T>::type VT;
    constexpr int W = Vec16<T>::W;
    const long long step = (long long)W * wr * kWave;
    long long r = r0 + (long long)W * ((long long)rw * kWave + lane);
    VT ua, za, va[NC], ub, zb, vn[NC];
#pragma unroll
    for (int e = 0; e < W; ++e) ua[e] = za[e] = ub[e] = zb[e] = T(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) va[c] = vn[c] = ua;
    auto load = [&](VT& uu, VT& zz, VT* vv, long long rr) {
      uu = ld16<T>(u + (rr - uoff));
      if constexpr (Z) zz = ld16<T>(z + (rr - zoff));
#pragma unroll
      for (int c = 0; c < NC; ++c) vv[c] = ld16_stream<T>(vb + (size_t)c * ldv + rr);
    };
    auto consume = [&](const VT& uu, const VT& zz, const VT* vv) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int e = 0; e < W; ++e) {
          ap[c] = fma((double)vv[c][e], (double)uu[e], ap[c]);
          if constexpr (Z) aq[c] = fma((double)vv[c][e], (double)zz[e], aq[c]);
        }
      }
    };
    if (r + W - 1 < r1) load(ua, za, va, r);
    while (r + W - 1 < r1) {
      long long rn = r + step;
      load(ub, zb, vn, (rn + W - 1 < r1) ? rn : r);
      consume(ua, za, va);
      r = rn;
      if (!(r + W - 1 < r1)) break;
      rn = r + step;
      load(ua, za, va, (rn + W - 1 < r1) ? rn : r);
      consume(ub, zb, vn);
      r = rn;
    }
    // the last rows of the block's range that do not fill a vector
    for (long long rr = r; rr < r1 && rr < r + W; ++rr) {
      const double uv = (double)u[rr - uoff];
      const double zv = Z ? (double)z[rr - zoff] : 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double v = (double)vb[(size_t)c * ldv + rr];
        ap[c] = fma(v, uv, ap[c]);
        if constexpr (Z) aq[c] = fma(v, zv, aq[c]);
      }
    }
  } else {
    // any alignment: element loads, U row steps
    constexpr int U = (NC >= 8) ? 1 : ((NC >= 4) ? 2 : 4);
    const long long step = (long long)wr * kWave;
    long long r = r0 + (long long)rw * kWave + lane;
    for (; r + (U - 1) * step < r1; r += U * step) {
      double uu[U], zz[U], vv[U][NC];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        uu[q] = (double)u[r + q * step - uoff];
        if constexpr (Z) zz[q] = (double)z[r + q * step - zoff];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
#pragma unroll
        for (int c = 0; c < NC; ++c) vv[q][c] = (double)vb[(size_t)c * ldv + r + q * step];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          ap[c] = fma(vv[q][c], uu[q], ap[c]);
          if constexpr (Z) aq[c] = fma(vv[q][c], zz[q], aq[c]);
        }
      }
    }
    for (; r < r1; r += step) {
      const double uv = (double)u[r - uoff];
      const double zv = Z ? (double)z[r - zoff] : 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double v = (double)vb[(size_t)c * ldv + r];
        ap[c] = fma(v, uv, ap[c]);
        if constexpr (Z) aq[c] = fma(v, zv, aq[c]);
      }
    }
  }
}

// The partial column group (nc < CPW columns, the last one) dispatches to the
// instantiation for its exact width.
template <int CPW, bool VEC, bool Z, typename T>
__device__ __forceinline__ void stream_group(int nc, const T* __restrict__ vb, long long ldv,
                                             const T* __restrict__ u, long long uoff,
                                             const T* __restrict__ z, long long zoff,
                                             long long r0, long long r1, int rw, int wr,
                                             int lane, double* ap, double* aq) {
  if (nc == CPW) {
    stream_cols<CPW, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq);
    return;
  }
  if constexpr (CPW > 1) {
    switch (nc) {
      case 1: stream_cols<1, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      case 2: if constexpr (CPW > 2) stream_cols<2, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      case 3: if constexpr (CPW > 3) stream_cols<3, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      case 4: if constexpr (CPW > 4) stream_cols<4, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      case 5: if constexpr (CPW > 5) stream_cols<5, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      case 6: if constexpr (CPW > 6) stream_cols<6, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      case 7: if constexpr (CPW > 7) stream_cols<7, VEC, Z, T>(vb, ldv, u, uoff, z, zoff, r0, r1, rw, wr, lane, ap, aq); break;
      default: break;
    }
  }
}

// The basis and A u in the element type of the step kernels.
template <typename T> __host__ __device__ T* basis(const Work& w);
template <> __host__ __device__ double* basis<double>(const Work& w) { return w.V; }
template <> __host__ __device__ float* basis<float>(const Work& w) { return w.V32; }
template <typename T> __host__ __device__ T* zvec(const Work& w);
template <> __host__ __device__ double* zvec<double>(const Work& w) { return w.z; }
template <> __host__ __device__ float* zvec<float>(const Work& w) { return w.z32; }

// Shared memory of the reduction (doubles): the wave partials of the older
// columns (wr rows of 2 ncol), or the totals and the grid-reduction scratch
// (2 ncol + max(threads, 2 ncol)), whichever is larger; then the fresh
// columns' partial sums (4 per wave).
__host__ __device__ __forceinline__ size_t fresh_lds_offset(int wr, int ncol) {
  const size_t nv = (size_t)2 * ncol;
  const size_t a = (size_t)wr * nv;
  const size_t b = nv + (nv > (size_t)kReduceThreads ? nv : (size_t)kReduceThreads);
  return a > b ? a : b;
}

// ZS: z is the block's own rows of A u in shared memory (zsh[r - r0]), formed
// by the fused operator apply, and so is u (ush[r - r0]) unless ush is null;
// sm: the shared memory of the reduction (the dynamic shared memory when
// null).
template <int CPW, bool VEC, bool Z, typename T, bool ZS = false>
__device__ __forceinline__ void reduce_body(
    Grid gr, const Work& w, long long n, int j, long long rows_per_block, int cpw, int wc, int wr,
    const T* __restrict__ Vraw, long long ldv_raw, const T* __restrict__ zraw,
    double* __restrict__ raw_out, double* sm = nullptr, const T* zsh = nullptr,
    const T* ush = nullptr) {
  extern __shared__ double dyn_lds[];
  double* lds = ZS ? sm : dyn_lds;
  const bool raw = (raw_out != nullptr);
  if (!ZS && !raw && !ctl_runs(w.ctl, j)) return;
  const T* __restrict__ V = raw ? Vraw : basis<T>(w);
  const long long ldv = raw ? ldv_raw : w.ldv;
  const int ncol = j + 1;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  // column split (small systems, w.red_csplit > 1): block bid takes row
  // block bid / cs and the columns [cb0, cb1) of part bid % cs; its partial
  // sums of the other columns are zero
  const int cs = (!ZS && !raw && w.red_csplit > 1) ? w.red_csplit : 1;
  const int cb = gr.bid % cs;
  const int cb0 = (int)((long long)ncol * cb / cs), cb1 = (int)((long long)ncol * (cb + 1) / cs);
  const long long r0 = (long long)(gr.bid / cs) * rows_per_block;
  const long long r1 = min(n, r0 + rows_per_block);
  const T* __restrict__ z = ZS ? zsh : (raw ? zraw : zvec<T>(w));
  const long long zoff = ZS ? r0 : 0;
  const T* __restrict__ u = (ZS && ush) ? ush : V + (size_t)j * ldv;
  const long long uoff = (ZS && ush) ? r0 : 0;
  // Without a column split, the columns the previous kernels have just
  // written, v_{j-1} and u_j, are summed first in a pass of their own by all
  // waves over the block's rows (a freshly written column read inside a
  // stream of many others slows the whole stream), and the column groups
  // below stream the older columns [0, f0) only.
  const int f0 = (cs == 1) ? (j >= 1 ? j - 1 : 0) : ncol;
  double* fr = lds + fresh_lds_offset(wr, ncol);   // [waves][4] fresh partial sums
  if (cs == 1) {
    double ap[2] = {0.0, 0.0}, aq[2] = {0.0, 0.0};
    stream_group<2, VEC, Z, T>(ncol - f0, V + (size_t)f0 * ldv, ldv, u, uoff, z, zoff, r0, r1, wave,
                               kReduceWaves, lane, ap, aq);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double sp = wave_sum(ap[c]);
      const double sq = wave_sum(aq[c]);
      if (lane == 0) {
        fr[wave * 4 + c] = sp;
        fr[wave * 4 + 2 + c] = sq;
      }
    }
  }
  const int cend = (cs == 1) ? f0 : cb1;
  const int nchunk = (cend - cb0 + cpw - 1) / cpw;
  const int cw = wave % wc;
  const int rw = wave / wc;
  if (rw < wr) {
    for (int ch = cw; ch < nchunk; ch += wc) {
      const int c0 = cb0 + ch * cpw;
      const int nc = min(cpw, cend - c0);
      double ap[CPW], aq[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) ap[c] = aq[c] = 0.0;
      stream_group<CPW, VEC, Z, T>(nc, V + (size_t)c0 * ldv, ldv, u, uoff, z, zoff, r0, r1, rw, wr,
                                   lane, ap, aq);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        if (c < nc) {
          const double sp = wave_sum(ap[c]);
          const double sq = wave_sum(aq[c]);
          if (lane == 0) {
            lds[(size_t)rw * 2 * ncol + c0 + c] = sp;
            lds[(size_t)rw * 2 * ncol + ncol + c0 + c] = sq;
          }
        }
      }
    }
  }
  __syncthreads();
  // the block's partial sums, written by wave 0 only (see grid_reduce_last)
  if (wave == 0) {
    double* part = w.part + (size_t)gr.bid * w.pstride;
    for (int v = lane; v < 2 * ncol; v += kWave) {
      const int col = v < ncol ? v : v - ncol;
      double acc = 0.0;
      if (col >= f0) {
        // a fresh column: the waves' sums in order
        const int k4 = (v < ncol ? 0 : 2) + (col - f0);
        for (int k = 0; k < kReduceWaves; ++k) acc += fr[k * 4 + k4];
      } else if (col >= cb0 && col < cb1) {
        for (int k = 0; k < wr; ++k) acc += lds[(size_t)k * 2 * ncol + v];
      }
      put_partial(part + v, acc);
    }
  }
  if (!raw) {
    // The group totals stay in w.gpart: every block of this iteration's
    // update kernel sums them and runs the small solve itself.
    group_reduce_last(w.part, w.gpart, w.pstride, w.tickets, 2 * ncol, lds, lds + 2 * ncol, gr);
    return;
  }
  if (!grid_reduce_last(w.part, w.gpart, w.pstride, w.tickets, 2 * ncol, lds, lds + 2 * ncol, gr))
    return;
  for (int v = threadIdx.x; v < 2 * ncol; v += blockDim.x) raw_out[v] = lds[v];
}

template <int CPW, bool VEC, bool Z, typename T>
__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(
    Work w, long long n, int j, long long rows_per_block, int cpw, int wc, int wr,
    const T* __restrict__ Vraw, long long ldv_raw, const T* __restrict__ zraw,
    double* __restrict__ raw_out) {
  reduce_body<CPW, VEC, Z, T>(hw_grid(), w, n, j, rows_per_block, cpw, wc, wr, Vraw, ldv_raw, zraw,
                              raw_out);
}

// Shared memory of the fused reduction: the wave partials; then the totals
// (2 ncol) followed by the grid-reduction scratch.
static size_t reduce_lds_bytes(const ReduceShape& s, int ncol) {
  return (fresh_lds_offset(s.wr, ncol) + 4 * kReduceWaves) * sizeof(double);
}

// Column groups of the reduction of iteration j: the older columns [0, j-1)
// (the fresh ones, v_{j-1} and u_j, have a pass of their own).
static ReduceShape reduce_shape(int j) { return reduce_columns(j >= 2 ? j - 1 : 1); }

// Blocks of `kernel` that are resident at once on the current device with
// `threads` threads and `lds` bytes of dynamic shared memory (cached); with
// kernel == nullptr, the number of compute units.
static int resident_blocks(const void* kernel, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  const auto key = std::make_tuple(dev, kernel, threads, lds);
  std::lock_guard<std::mutex> g(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per = 0;
  if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  // kernel == nullptr: the number of CUs
  if (kernel == nullptr) per = 1;
  else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) != hipSuccess ||
           per < 1)
    per = 1;
  const int r = cus * per;
  cache[key] = r;
  return r;
}

template <typename T>
using ReduceKernel = void (*)(Work, long long, int, long long, int, int, int, const T*, long long,
                              const T*, double*);

template <typename T>
static ReduceKernel<T> pick_reduce(int tcpw, bool vec, bool z) {
  switch (tcpw * 4 + (vec ? 2 : 0) + (z ? 1 : 0)) {
#define IGS_RED_CASE(C, VV, ZZ) \
  case C * 4 + VV * 2 + ZZ: return reduce_kernel<C, VV, ZZ, T>;
#define IGS_RED_CASES(C) \
  IGS_RED_CASE(C, 0, 0) IGS_RED_CASE(C, 0, 1) IGS_RED_CASE(C, 1, 0) IGS_RED_CASE(C, 1, 1)
    IGS_RED_CASES(1) IGS_RED_CASES(2) IGS_RED_CASES(4) IGS_RED_CASES(8)
#undef IGS_RED_CASES
#undef IGS_RED_CASE
    default: return nullptr;
  }
}

template <typename T>
static hipError_t reduce_dispatch(const Work& w, long long n, int j, bool with_z, const T* Vraw,
                                  long long ldv_raw, const T* zraw, double* raw_out,
                                  hipStream_t s, int* nblocks_out) {
  const int ncol = j + 1;
  ReduceShape sh = reduce_shape(j);
  const size_t lds = reduce_lds_bytes(sh, ncol);
  // 16-byte row vectors need a leading dimension of whole vectors and
  // 16-byte aligned columns
  const T* Vp = raw_out ? Vraw : basis<T>(w);
  const T* zp = raw_out ? zraw : zvec<T>(w);
  const long long ldv = raw_out ? ldv_raw : w.ldv;
  const bool vec = (ldv % Vec16<T>::W == 0) && (reinterpret_cast<uintptr_t>(Vp) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(zp) % 16 == 0);
  ReduceKernel<T> k = pick_reduce<T>(sh.tcpw, vec, with_z);
  if (k == nullptr) return hipErrorInvalidValue;
  // One round of resident blocks.  The grid (and so the summation order) is
  // the one of the variant with z, so that the tail iteration, which has no
  // z, forms V^T u exactly as the others do.
  int cap = resident_blocks(reinterpret_cast<const void*>(pick_reduce<T>(sh.tcpw, vec, true)),
                            kReduceThreads, lds);
  if (cap > kMaxBlocks) cap = kMaxBlocks;
  // with one or two columns a block streams little: one block per CU keeps
  // the fixed per-block costs (partials, arrival counters) small
  if (sh.tcpw <= 2) {
    const int cus = resident_blocks(nullptr, 0, 0);
    if (cap > cus) cap = cus;
  }
  if (w.tune && (w.tune[j] & 1) && cap > 1) cap /= 2;
  reduce_rows(sh, n, cap);
  // A small system with many columns (allowed by the solve): split the
  // columns over several blocks per row block, at least 8 columns each, so
  // that about half the CUs take part.
  int csplit = 1;
  size_t lds_launch = lds;
  ReduceKernel<T> kl = k;
  if (!raw_out && w.col_split) {
    const int cus = resident_blocks(nullptr, 0, 0);
    const int want = (cus / 2) / sh.nblocks;
    csplit = std::min((ncol + 7) / 8, want);
    if (csplit > 1) {
      ReduceShape sc = reduce_columns((ncol + csplit - 1) / csplit);
      sc.rows_per_block = sh.rows_per_block;
      sc.nblocks = sh.nblocks * csplit;
      sh = sc;
      lds_launch = reduce_lds_bytes(sh, ncol);
      kl = pick_reduce<T>(sh.tcpw, vec, with_z);
      if (kl == nullptr) return hipErrorInvalidValue;
    } else {
      csplit = 1;
    }
  }
  if (nblocks_out) *nblocks_out = sh.nblocks;
  Work wa = w;
  wa.red_csplit = csplit;
  long long na = n, rpb = sh.rows_per_block, ldva = ldv_raw;
  int ja = j, cpw = sh.cpw, wc = sh.wc, wr = sh.wr;
  const T* va = Vraw;
  const T* za = zraw;
  double* oa = raw_out;
  void* args[] = {&wa, &na, &ja, &rpb, &cpw, &wc, &wr, &va, &ldva, &za, &oa};
  return hipLaunchKernel(reinterpret_cast<const void*>(kl), dim3(sh.nblocks), dim3(kReduceThreads),
                         args, lds_launch, s);
}

hipError_t launch_reduce(const Work& w, long long n, int j, bool with_z, hipStream_t s,
                         int* nblocks_out) {
  if (w.fp32)
    return reduce_dispatch<float>(w, n, j, with_z, nullptr, 0, nullptr, nullptr, s, nblocks_out);
  return reduce_dispatch<double>(w, n, j, with_z, nullptr, 0, nullptr, nullptr, s, nblocks_out);
}

hipError_t launch_reduce_raw(const double* V, long long ldv, long long n, int j, const double* z,
                             double* part, double* gpart, int pstride, unsigned* tickets,
                             double* out, hipStream_t s) {
  Work w{};
  w.part = part;
  w.gpart = gpart;
  w.pstride = pstride;
  w.tickets = tickets;
  return reduce_dispatch<double>(w, n, j, z != nullptr, V, ldv, z, out, s, nullptr);
}

// ---------------------------------------------------------------------------
// Operator apply fused into the reduction: A u, then [V_{0:j}, u]^T [u, A u]
// ---------------------------------------------------------------------------
//
// With the operator in ELL form, each block of the fused reduction first forms
// z = A u for its own rows, keeps them in shared memory for V^T z and stores
// them for the update kernel; then it runs the reduction of reduce_body on the
// same grid.  Against the operator apply and the reduction as two kernels,
// u is read once and z is never read back from device memory, and the
// iteration has one launch less.  z is bit-identical to the ELL (and CSR)
// kernel's: every row's products and additions are theirs, in their order,
// with contraction off; the reduction then adds the same values in the same
// order, so its sums are bit-identical too.

// R consecutive rows r .. r+R-1 of z = A x from the column-major ELL form
// (entry slot k of row r at k n + r; K <= 8 slots): each slot's column indices
// and values are read as one vector of R.  D16: the indices are 16-bit
// offsets from the row (col - r), padding 0.  Needs n and r multiples of R
// and arrays aligned to their vectors.
template <typename T, int R, bool D16>
__device__ __forceinline__ void ell_rowsR(const void* __restrict__ idx, const T* __restrict__ val,
                                          long long n, int K, const T* __restrict__ x,
                                          long long r, T* out) {
#pragma clang fp contract(off)
  typedef typename std::conditional<D16, short, int>::type I;
  typedef I IR __attribute__((ext_vector_type(R)));
  typedef T AR __attribute__((ext_vector_type(R)));
  const I* __restrict__ col = static_cast<const I*>(idx);
  IR c[8];
  AR v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < K) {
      c[k] = *reinterpret_cast<const IR*>(col + (long long)k * n + r);
      v[k] = *reinterpret_cast<const AR*>(val + (long long)k * n + r);
    } else {
      c[k] = IR(0);
      v[k] = AR(0);
    }
  }
  T g[8][R];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int i = 0; i < R; ++i)
      g[k][i] = D16 ? x[r + i + (long long)c[k][i]] : x[(long long)c[k][i]];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    T p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = v[k][i] * g[k][i];
    const T q0 = (p[0] + p[1]) + (p[2] + p[3]);
    const T q1 = (p[4] + p[5]) + (p[6] + p[7]);
    out[i] = q0 + q1;
  }
}

template <int CPW, typename T, bool D16>
__global__ __launch_bounds__(kReduceThreads) void opreduce_kernel(
    Work w, long long n, int j, long long rows_per_block, int cpw, int wc, int wr, int ell_k,
    const void* __restrict__ ell_idx, const T* __restrict__ ell_val, int u_lds) {
  extern __shared__ double lds[];
  if (!ctl_runs(w.ctl, j)) return;
  const Grid gr = hw_grid();
  const long long r0 = (long long)gr.bid * rows_per_block;
  const long long r1 = min(n, r0 + rows_per_block);
  // shared memory: the block's rows of z and (u_lds) of u, rows_per_block
  // values each (a multiple of 256), then the reduction's own
  T* zs = reinterpret_cast<T*>(lds);
  T* us = u_lds ? zs + rows_per_block : nullptr;
  double* sm = lds + (size_t)rows_per_block * (u_lds ? 2 : 1) * sizeof(T) / sizeof(double);
  const T* __restrict__ u = basis<T>(w) + (size_t)j * w.ldv;
  T* __restrict__ zg = zvec<T>(w);
  // Two rows per thread and step, each entry slot's values read as one vector
  // of two (two rows of doubles: 116.1 -> 113.9 us per launch against four
  // at 128^3; of floats: 31.6 -> 28.9 us against four at 96^3).
  typedef T A2 __attribute__((ext_vector_type(2)));
  for (long long r = r0 + 2 * (long long)threadIdx.x; r < r1; r += 2LL * kReduceThreads) {
    T out[2];
    ell_rowsR<T, 2, D16>(ell_idx, ell_val, n, ell_k, u, r, out);
    // the block's own rows of u (also among the gathers) for every column
    // group of the reduction, which would otherwise read them again from
    // device memory
    if (us != nullptr) *reinterpret_cast<A2*>(us + (r - r0)) = *reinterpret_cast<const A2*>(u + r);
    A2 o;
    o[0] = out[0];
    o[1] = out[1];
    *reinterpret_cast<A2*>(zs + (r - r0)) = o;
    __builtin_nontemporal_store(o, reinterpret_cast<A2*>(zg + r));   // see st16
  }
  __syncthreads();
  reduce_body<CPW, true, true, T, true>(gr, w, n, j, rows_per_block, cpw, wc, wr, nullptr, 0,
                                        nullptr, nullptr, sm, zs, us);
}

template <typename T>
using OpReduceKernel = void (*)(Work, long long, int, long long, int, int, int, int, const void*,
                                const T*, int);

template <typename T>
static OpReduceKernel<T> pick_opreduce(int tcpw, bool d16) {
  switch (tcpw * 2 + (d16 ? 1 : 0)) {
    case 2: return opreduce_kernel<1, T, false>;
    case 3: return opreduce_kernel<1, T, true>;
    case 4: return opreduce_kernel<2, T, false>;
    case 5: return opreduce_kernel<2, T, true>;
    case 8: return opreduce_kernel<4, T, false>;
    case 9: return opreduce_kernel<4, T, true>;
    case 16: return opreduce_kernel<8, T, false>;
    case 17: return opreduce_kernel<8, T, true>;
    default: return nullptr;
  }
}

// Largest share of a block's rows of z kept in shared memory (bytes).  Its
// rows of u are kept there too when both fit.
constexpr size_t kFusedZBytes = 128 * 1024;

// Dynamic shared memory a block may use on the current device (cached).
static size_t max_lds_per_block() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(mu);
  const auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v < 0)
    v = 0;
  cache[dev] = (size_t)v;
  return (size_t)v;
}

// The launch of the fused kernel for iteration j, or nblocks = 0 when the
// operator apply and the reduction must run as two kernels: no ELL form,
// n not a multiple of 4, arrays the vector loads cannot take, or a block's
// rows of z beyond the shared memory.  The grid is the separate reduction's,
// and the fused kernel must hold all of it resident at once.
struct FusedLaunch {
  const void* kernel = nullptr;
  ReduceShape sh{};
  size_t lds = 0;
  int u_lds = 0;
  const void* idx = nullptr;   // ELL column indices: 32-bit, or 16-bit offsets
  int nblocks = 0;
};

template <typename T>
static FusedLaunch opreduce_plan(const Op& op, const Work& w, long long n, int j) {
  FusedLaunch f;
  const T* ev = ell_vals<T>(op);
  const T* V = basis<T>(w);
  const T* z = zvec<T>(w);
  if (op.dense || op.ell_k <= 0 || op.rpg != 0 || ev == nullptr || n % 4 != 0) return f;
  if (reinterpret_cast<uintptr_t>(op.ell_col) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(ev) % (4 * sizeof(T)) != 0 ||
      reinterpret_cast<uintptr_t>(z) % (4 * sizeof(T)) != 0 ||
      reinterpret_cast<uintptr_t>(V) % 16 != 0 || w.ldv % Vec16<T>::W != 0)
    return f;
  // the column indices as 16-bit offsets from the row where they exist
  const bool d16 = op.ell_dcol != nullptr && reinterpret_cast<uintptr_t>(op.ell_dcol) % 16 == 0;
  const int ncol = j + 1;
  ReduceShape sh = reduce_shape(j);
  const size_t red_lds = reduce_lds_bytes(sh, ncol);
  // the separate reduction's grid (reduce_dispatch)
  int cap = resident_blocks(reinterpret_cast<const void*>(pick_reduce<T>(sh.tcpw, true, true)),
                            kReduceThreads, red_lds);
  if (cap > kMaxBlocks) cap = kMaxBlocks;
  if (sh.tcpw <= 2) {
    const int cus = resident_blocks(nullptr, 0, 0);
    if (cap > cus) cap = cus;
  }
  if (w.tune && (w.tune[j] & 1) && cap > 1) cap /= 2;
  reduce_rows(sh, n, cap);
  const size_t zbytes = (size_t)sh.rows_per_block * sizeof(T);
  if (zbytes > kFusedZBytes) return f;
  const void* k = reinterpret_cast<const void*>(pick_opreduce<T>(sh.tcpw, d16));
  if (k == nullptr) return f;
  const size_t cap_lds = max_lds_per_block();
  const int u_lds = (2 * zbytes + red_lds <= cap_lds) ? 1 : 0;
  const size_t lds = (u_lds ? 2 : 1) * zbytes + red_lds;
  if (lds > cap_lds) return f;
  if (resident_blocks(k, kReduceThreads, lds) < sh.nblocks) return f;
  f.kernel = k;
  f.sh = sh;
  f.lds = lds;
  f.u_lds = u_lds;
  f.idx = d16 ? static_cast<const void*>(op.ell_dcol) : static_cast<const void*>(op.ell_col);
  f.nblocks = sh.nblocks;
  return f;
}

bool opreduce_fits(const Op& op, const Work& w, long long n, int j) {
  return (w.fp32 ? opreduce_plan<float>(op, w, n, j) : opreduce_plan<double>(op, w, n, j))
             .nblocks > 0;
}

template <typename T>
static hipError_t opreduce_launch(const Op& op, const Work& w, long long n, int j, hipStream_t s,
                                  int* nblocks_out) {
  const FusedLaunch f = opreduce_plan<T>(op, w, n, j);
  if (f.nblocks == 0) return hipErrorInvalidValue;
  if (nblocks_out) *nblocks_out = f.nblocks;
  Work wa = w;
  long long na = n, rpb = f.sh.rows_per_block;
  int ja = j, cpw = f.sh.cpw, wc = f.sh.wc, wr = f.sh.wr, k = op.ell_k;
  const void* idx = f.idx;
  const T* val = ell_vals<T>(op);
  int ul = f.u_lds;
  void* args[] = {&wa, &na, &ja, &rpb, &cpw, &wc, &wr, &k, &idx, &val, &ul};
  return hipLaunchKernel(f.kernel, dim3(f.nblocks), dim3(kReduceThreads), args, f.lds, s);
}

hipError_t launch_opreduce(const Op& op, const Work& w, long long n, int j, hipStream_t s,
                           int* nblocks_out) {
  if (w.fp32) return opreduce_launch<float>(op, w, n, j, s, nblocks_out);
  return opreduce_launch<double>(op, w, n, j, s, nblocks_out);
}

// ---------------------------------------------------------------------------
// The fused reduction without allocation
// ---------------------------------------------------------------------------
//
// Its per-block partial sums, group totals and arrival counters live in one
// static device array of the library instead of a workspace.  The array's
// name is a host-side stand-in in host code: its address on each device is
// taken once with hipGetSymbolAddress and only that address reaches kernels.

constexpr int kNoAllocStride = 2 * kNoAllocMaxCols;   // doubles per partial-sum row
constexpr size_t kNoAllocPartDoubles = (size_t)kMaxBlocks * kNoAllocStride;
constexpr size_t kNoAllocGroupDoubles = (size_t)kMaxGroups * kNoAllocStride;
constexpr size_t kNoAllocCounterDoubles = 64;          // kMaxGroups + 1 counters, padded
constexpr size_t kNoAllocDoubles = kNoAllocPartDoubles + kNoAllocGroupDoubles + kNoAllocCounterDoubles;
static_assert((kMaxGroups + 1) * sizeof(unsigned) <= kNoAllocCounterDoubles * sizeof(double),
              "counter area too small");
static_assert(kNoAllocDoubles * sizeof(double) == kNoAllocBytes, "scratch size mismatch");

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kNoAllocMaxDevices = 64;

struct NoAllocDevice {
  std::once_flag once;
  hipError_t err = hipSuccess;
  double* ptr = nullptr;   // the device address of `scratch` on this device
};
static NoAllocDevice g_noalloc[kNoAllocMaxDevices];

// Zero the arrival counters (a kernel, not a memset, so that the call can be
// recorded into a HIP graph and replayed).
__global__ void clear_counters_kernel(unsigned* c, int count) {
  if ((int)threadIdx.x < count) c[threadIdx.x] = 0u;
}

hipError_t launch_reduce_noalloc(const double* V, long long ldv, long long n, int j,
                                 const double* z, double* out, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  NoAllocDevice& d = g_noalloc[dev];
  // Once per device, with that device current: the array's address there, and
  // the occupancy queries of every reduction shape this entry point can
  // launch, so that later calls only queue kernels.
  std::call_once(d.once, [&] {
    void* p = nullptr;
    d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (d.err != hipSuccess) return;
    d.ptr = static_cast<double*>(p);
    for (int ncol = 1; ncol <= kNoAllocMaxCols; ++ncol) {
      const ReduceShape sh = reduce_shape(ncol - 1);
      const size_t lds = reduce_lds_bytes(sh, ncol);
      for (int vec = 0; vec < 2; ++vec)
        (void)resident_blocks(reinterpret_cast<const void*>(pick_reduce<double>(sh.tcpw, vec, true)),
                              kReduceThreads, lds);
    }
    (void)resident_blocks(nullptr, 0, 0);
  });
  if (d.err != hipSuccess) return d.err;
  if (d.ptr == nullptr) return hipErrorInvalidSymbol;
  double* part = d.ptr;
  double* gpart = d.ptr + kNoAllocPartDoubles;
  unsigned* tickets = reinterpret_cast<unsigned*>(d.ptr + kNoAllocPartDoubles + kNoAllocGroupDoubles);
  hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(128), 0, s, tickets, kMaxGroups + 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  Work w{};
  w.part = part;
  w.gpart = gpart;
  w.pstride = kNoAllocStride;
  w.tickets = tickets;
  return reduce_dispatch<double>(w, n, j, z != nullptr, V, ldv, z, out, s, nullptr);
}

// ---------------------------------------------------------------------------
// Basis update: one pass over V_{0:j}
// ---------------------------------------------------------------------------

// Shared memory of the update kernel for iteration j: the reduction totals
// (2 (j+1)), the small-solve scratch (7 (j+2)) and the staged T and H.
__host__ __device__ __forceinline__ size_t update_lds_doubles(int j) {
  return (size_t)2 * (j + 1) + (size_t)7 * (j + 2) + stage_count(j);
}

// Rows of one tile of the update: every thread owns NV 16-byte row vectors
// (2 NV rows of doubles or 4 NV of floats), so a block reads each column of V
// in runs of NV x 4 KB.  Longer runs per column stream faster from HBM (about
// 6.2 TB/s with 8 KB runs against 6.8 with 16 KB on the 2M-row basis; with
// 32 KB runs and the column loads pipelined, the 2M-row update takes 85.7
// against 91.1 us).
template <typename T, int NV = 2>
__host__ __device__ constexpr long long update_tile_rows() {
  return (long long)NV * Vec16<T>::W * kUpdateThreads;
}

// The coefficients of the two-reduce second sweep for the vector in column j
// (every block; the publisher also adds them to the first-sweep
// coefficients of column j-1): t = T_j P[0:j], from LDS when T is staged.
__device__ void correct_coefs(const Work& w, int j, const double* P, double* sm, bool pub) {
  double* st = sm;
  double* stg = sm + 7 * (j + 2);
  // staged when the update kernel's shared memory holds the staging area
  if (stage_count(j) > 0) {
    stage_copy(stg, w.T, tri_row(j));
    __syncthreads();
    tri_matvec<true>(stg, P, st, j);
  } else {
    tri_matvec<false>(w.T, P, st, j);
  }
  __syncthreads();
  if (pub)
    for (int i = threadIdx.x; i < j; i += blockDim.x) w.coef_r1[i] += st[i];
}

template <bool HAS_T, bool VEC, typename T, int NV>
__device__ __forceinline__ void update_body(
    Grid gr, const Work& w, long long n, int j, int ngroups, T* __restrict__ Vraw,
    long long ldv_raw, const T* __restrict__ zraw, const double* __restrict__ traw,
    const double* __restrict__ r1raw, double igraw, int raw) {
  // raw: 1 = step kernel on caller buffers, 2 = two-reduce second sweep
  typedef typename Vec16<T>::type VT;
  constexpr int W = Vec16<T>::W;
  constexpr int R = NV * W;  // rows per thread and tile
  extern __shared__ double sdyn[];
  double* sP = sdyn;                 // V_{0:j}^T u and u^T u
  double* sQ = sdyn + (j + 1);       // V_{0:j}^T z and u^T z
  double* sm = sdyn + 2 * (j + 1);   // small-solve scratch; t at sm, r1 at sm + 2 (j+2)
  const double* t = sm;
  const double* r1 = sm + 2 * (j + 2);
  int mode;
  double ig;
  T* __restrict__ V;
  long long ldv;
  const T* __restrict__ z;
  if (raw == 1) {
    mode = kUpdNormal;
    ig = igraw;
    V = Vraw;
    ldv = ldv_raw;
    z = zraw;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
      if (i < j) sm[i] = traw[i];
      sm[2 * (j + 2) + i] = r1raw[i];
    }
    __syncthreads();
  } else {
    if (!ctl_runs(w.ctl, j)) return;
    V = basis<T>(w);
    ldv = w.ldv;
    z = zvec<T>(w);
    // the reduction totals: the group rows it left, summed in a fixed order
    for (int v = threadIdx.x; v < 2 * (j + 1); v += blockDim.x) {
      double g8[8];
#pragma unroll
      for (int g = 0; g < 8; ++g) g8[g] = (g < ngroups) ? w.gpart[(size_t)g * w.pstride + v] : 0.0;
      double acc = g8[0];
#pragma unroll
      for (int g = 1; g < 8; ++g) acc += g8[g];
      sdyn[v] = acc;
    }
    __syncthreads();
    const bool pub = (gr.bid == 0);
    if (raw == 2) {
      correct_coefs(w, j, sP, sm, pub);
      mode = kUpdCorrect;
      ig = 1.0;
    } else {
      const bool tail = (j >= w.ctl->m);
      const StepCoefs c =
          (stage_count(j) > 0)
              ? small_solve<kSolveStaged>(w, n, j, tail, sP, sQ, sm, pub)
              : (w.pre_on ? small_solve<kSolvePre>(w, n, j, tail, sP, sQ, sm, pub)
                          : small_solve<kSolveGlobal>(w, n, j, tail, sP, sQ, sm, pub));
      mode = c.mode;
      ig = c.ig;
      if (mode == kUpdNone) return;
    }
  }
  const bool need_r = (mode == kUpdNormal);
  const bool fallback = (mode == kUpdFallback);
  const bool unscaled = fallback || (mode == kUpdCorrect);   // w = u - V t, stored as is
  const double rj = need_r ? r1[j] : 0.0;
  T* __restrict__ vj = V + (size_t)j * ldv;
  T* __restrict__ un = V + (size_t)(j + 1) * ldv;
  double s2 = 0.0;  // ||w||^2 partial (fallback only)
  if constexpr (NV == 0) {
    // Column split, for systems too small to give every CU a tile of the
    // row-vector pass: a tile of 64 W rows per block, each of the 4 waves
    // forms the partial sums of its quarter of the columns for every row of
    // the tile (8 loads in flight per lane), and wave 0 adds the quarters in
    // order and writes.  Four times the blocks, a quarter of the column
    // batches on each block's latency chain.
    static_assert(VEC, "the column split takes 16-byte row vectors");
    constexpr int kNw = kUpdateThreads / kWave;
    constexpr long long kTileS = (long long)kWave * W;
    __shared__ double pa[kNw][kTileS], pb[kNw][kTileS];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int c0 = (int)((long long)j * wave / kNw), c1 = (int)((long long)j * (wave + 1) / kNw);
    const long long ntiles = (n + kTileS - 1) / kTileS;
    for (long long tile = gr.bid; tile < ntiles; tile += gr.nb) {
      const long long p = tile * kTileS + (long long)W * lane;
      const bool full = p + W <= n;
      double a[W], b[W];
#pragma unroll
      for (int e = 0; e < W; ++e) a[e] = b[e] = 0.0;
      auto use = [&](const double* v, int c) {
        const double tc = HAS_T ? t[c] : 0.0;
        const double rc = r1[c];
#pragma unroll
        for (int e = 0; e < W; ++e) {
          if (HAS_T) a[e] = fma(v[e], tc, a[e]);
          b[e] = fma(v[e], rc, b[e]);
        }
      };
      int c = c0;
      if (full) {
        for (; c + 8 <= c1; c += 8) {
          VT v[8];
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) v[cc] = ld16_stream<T>(V + (size_t)(c + cc) * ldv + p);
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) {
            double d[W];
#pragma unroll
            for (int e = 0; e < W; ++e) d[e] = (double)v[cc][e];
            use(d, c + cc);
          }
        }
        for (; c < c1; ++c) {
          const VT v = ld16_stream<T>(V + (size_t)c * ldv + p);
          double d[W];
#pragma unroll
          for (int e = 0; e < W; ++e) d[e] = (double)v[e];
          use(d, c);
        }
      } else {
        for (; c < c1; ++c) {
          double d[W];
#pragma unroll
          for (int e = 0; e < W; ++e) d[e] = (p + e < n) ? (double)V[(size_t)c * ldv + p + e] : 0.0;
          use(d, c);
        }
      }
#pragma unroll
      for (int e = 0; e < W; ++e) {
        pa[wave][W * lane + e] = a[e];
        pb[wave][W * lane + e] = b[e];
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const long long r = p + e;
          if (r >= n) continue;
          double sa = pa[0][W * lane + e], sb = pb[0][W * lane + e];
#pragma unroll
          for (int q = 1; q < kNw; ++q) {
            sa += pa[q][W * lane + e];
            sb += pb[q][W * lane + e];
          }
          if (unscaled) {
            const double wv = (double)vj[r] - sa;
            vj[r] = (T)wv;
            s2 = fma(wv, wv, s2);
          } else {
            const double v = ((double)vj[r] - sa) * ig;
            vj[r] = (T)v;
            if (need_r) un[r] = (T)((double)z[r] * ig - sb - v * rj);
          }
        }
      }
      __syncthreads();
    }
  } else {
  constexpr long long kTile = update_tile_rows<T, NV>();
  const long long ntiles = (n + kTile - 1) / kTile;
  for (long long tile = gr.bid; tile < ntiles; tile += gr.nb) {
    if constexpr (VEC) {
      // Full tile: the thread owns the row vectors at p_k = W t + k W
      // kUpdateThreads; V is streamed with 16-byte non-temporal loads, CB
      // columns at a time (8 loads in flight per thread); products and sums
      // in FP64, each row's over the columns in order.
      constexpr int CB = (NV >= 4) ? 2 : 8 / NV;
      const long long tb = tile * kTile;
      if (tb + kTile <= n) {
        long long p[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k)
          p[k] = tb + (long long)W * threadIdx.x + (long long)k * W * kUpdateThreads;
        double a[NV][W], b[NV][W];
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
          for (int e = 0; e < W; ++e) a[k][e] = b[k][e] = 0.0;
        auto use = [&](const VT* v, int c) {
          const double tc = HAS_T ? t[c] : 0.0;
          const double rc = r1[c];
#pragma unroll
          for (int k = 0; k < NV; ++k) {
#pragma unroll
            for (int e = 0; e < W; ++e) {
              if (HAS_T) a[k][e] = fma((double)v[k][e], tc, a[k][e]);
              b[k][e] = fma((double)v[k][e], rc, b[k][e]);
            }
          }
        };
        int c = 0;
        if constexpr (NV >= 8) {
          // Two register stages of one column each, alternating roles: the
          // next column's loads are issued before the FMAs of the current
          // one (without a next column the current one is loaded again and
          // not used, so the loads stay unconditional).
          auto load = [&](VT* v, int cb) {
            const T* vc = V + (size_t)cb * ldv;
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = ld16_stream<T>(vc + p[k]);
          };
          if (j >= 1) {
            VT va[NV], vb[NV];
            load(va, 0);
            while (true) {
              load(vb, (c + 1 < j) ? c + 1 : c);
              use(va, c);
              ++c;
              if (c >= j) break;
              load(va, (c + 1 < j) ? c + 1 : c);
              use(vb, c);
              ++c;
              if (c >= j) break;
            }
          }
        }
        for (; c + CB <= j; c += CB) {
          VT v[CB][NV];
#pragma unroll
          for (int cc = 0; cc < CB; ++cc) {
            const T* vc = V + (size_t)(c + cc) * ldv;
#pragma unroll
            for (int k = 0; k < NV; ++k) v[cc][k] = ld16_stream<T>(vc + p[k]);
          }
#pragma unroll
          for (int cc = 0; cc < CB; ++cc) use(v[cc], c + cc);
        }
        for (; c < j; ++c) {
          const T* vc = V + (size_t)c * ldv;
          VT v[NV];
#pragma unroll
          for (int k = 0; k < NV; ++k) v[k] = ld16_stream<T>(vc + p[k]);
          use(v, c);
        }
        VT uu[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) uu[k] = ld16<T>(vj + p[k]);
        if (unscaled) {
#pragma unroll
          for (int k = 0; k < NV; ++k) {
            VT o;
#pragma unroll
            for (int e = 0; e < W; ++e) {
              const double wv = (double)uu[k][e] - a[k][e];
              o[e] = (T)wv;
              s2 = fma(wv, wv, s2);
            }
            st16<T>(vj + p[k], o);
          }
        } else {
          // v_j over the loaded u; a then holds v_j for the u_{j+1} rows
#pragma unroll
          for (int k = 0; k < NV; ++k) {
            VT o;
#pragma unroll
            for (int e = 0; e < W; ++e) {
              a[k][e] = ((double)uu[k][e] - a[k][e]) * ig;
              o[e] = (T)a[k][e];
            }
            st16<T>(vj + p[k], o);
          }
          if (need_r) {
            VT zz[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) zz[k] = ld16<T>(z + p[k]);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
              VT o;
#pragma unroll
              for (int e = 0; e < W; ++e)
                o[e] = (T)((double)zz[k][e] * ig - b[k][e] - a[k][e] * rj);
              st16<T>(un + p[k], o);
            }
          }
        }
        continue;
      }
    }
    // element path (partial tiles, or any alignment): R rows per thread,
    // taken 4 at a time (rows tile + tid + k kUpdateThreads), with 4 columns
    // of loads in flight before their FMAs
#pragma unroll 1
    for (int h = 0; h < R; h += 4) {
      const long long base = tile * kTile + threadIdx.x + (long long)h * kUpdateThreads;
      double at[4], ar[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) at[k] = ar[k] = 0.0;
      const bool full = base + 3LL * kUpdateThreads < n;
      if (full) {
        int c = 0;
        for (; c + 4 <= j; c += 4) {
          double vv[4][4];
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const T* __restrict__ vc = V + (size_t)(c + cc) * ldv + base;
#pragma unroll
            for (int k = 0; k < 4; ++k) vv[cc][k] = (double)vc[k * kUpdateThreads];
          }
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            const double tc = HAS_T ? t[c + cc] : 0.0;
            const double rc = r1[c + cc];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              if (HAS_T) at[k] = fma(vv[cc][k], tc, at[k]);
              ar[k] = fma(vv[cc][k], rc, ar[k]);
            }
          }
        }
        for (; c < j; ++c) {
          const T* __restrict__ vc = V + (size_t)c * ldv + base;
          const double tc = HAS_T ? t[c] : 0.0;
          const double rc = r1[c];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double v = (double)vc[k * kUpdateThreads];
            if (HAS_T) at[k] = fma(v, tc, at[k]);
            ar[k] = fma(v, rc, ar[k]);
          }
        }
      } else {
        for (int c = 0; c < j; ++c) {
          const T* __restrict__ vc = V + (size_t)c * ldv + base;
          const double tc = HAS_T ? t[c] : 0.0;
          const double rc = r1[c];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (base + k * kUpdateThreads < n) {
              const double v = (double)vc[k * kUpdateThreads];
              if (HAS_T) at[k] = fma(v, tc, at[k]);
              ar[k] = fma(v, rc, ar[k]);
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const long long r = base + k * kUpdateThreads;
        if (r < n) {
          if (unscaled) {
            const double wv = (double)vj[r] - at[k];
            vj[r] = (T)wv;
            s2 = fma(wv, wv, s2);
          } else {
            const double v = ((double)vj[r] - at[k]) * ig;
            vj[r] = (T)v;
            if (need_r) un[r] = (T)((double)z[r] * ig - ar[k] - v * rj);
          }
        }
      }
    }
  }
  }
  if (!fallback) return;
  // Lagged norm cancelled: w = u - V t is stored unnormalised; its explicit
  // norm comes from a grid reduction (group totals in rows 8.. of gpart, so
  // that the reduction totals in rows 0..7 stay intact for blocks that start
  // later) and finishes column j-1 in the last block.
  __shared__ double red[kUpdateThreads / kWave];
  __shared__ double tot[1];
  __shared__ double scr[kUpdateThreads];
  s2 = wave_sum(s2);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int k = 0; k < kUpdateThreads / kWave; ++k) acc += red[k];
    put_partial(w.part + (size_t)gr.bid * w.pstride, acc);
  }
  // (the last block reads the column block 0 stored in this launch: full fences)
  if (!grid_reduce_last(w.part, w.gpart + (size_t)8 * w.pstride, w.pstride, w.tickets, 1, tot, scr,
                        gr, true))
    return;
  const double gamma = sqrt(tot[0]);
  // scratch in shared memory: the column (as the publisher stored it), the
  // rotations and g[j-1]
  double* hcol = sm + (j + 2);
  double* fcs = sm + 5 * (j + 2);
  double* fsn = sm + 6 * (j + 2);
  __shared__ double s_gc;
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    hcol[i] = w.H[hess_col(j - 1) + i];
    if (i < j - 1) {
      fcs[i] = w.cs[i];
      fsn[i] = w.sn[i];
    }
  }
  if (threadIdx.x == 0) s_gc = w.g[j - 1];
  __syncthreads();
  const int brk = finish_column(w, j, hcol, gamma, fcs, fsn, s_gc, n);
  if (threadIdx.x == 0) {
    Ctl* c = w.ctl;
    c->J = j;
    c->end_iter = j;
    c->fallbacks += 1;
    if (brk) {
      c->status = kBreakdown;
      c->breakdowns += 1;
    } else {
      c->status = kLagnorm;
    }
    c->mode = kUpdNone;
  }
}

// With four row vectors of doubles, four blocks per CU (at most 128 VGPRs)
// give one tile to each block on the 2M-row basis.
template <bool HAS_T, bool VEC, typename T, int NV>
__global__ __launch_bounds__(kUpdateThreads)
__attribute__((amdgpu_waves_per_eu((NV == 4 && sizeof(T) == 8) ? 4 : 1))) void update_kernel(
    Work w, long long n, int j, int ngroups, T* __restrict__ Vraw, long long ldv_raw,
    const T* __restrict__ zraw, const double* __restrict__ traw,
    const double* __restrict__ r1raw, double igraw, int raw) {
  update_body<HAS_T, VEC, T, NV>(hw_grid(), w, n, j, ngroups, Vraw, ldv_raw, zraw, traw, r1raw,
                                 igraw, raw);
}

// Tiles of update_tile_rows<T>() rows, one round of resident blocks striding
// over them (so that every block runs the small solve once), capped so that
// the per-block partials of the fallback path fit their buffer.
static unsigned update_grid(const void* kernel, long long n, long long tile_rows, size_t lds) {
  const long long tiles = (n + tile_rows - 1) / tile_rows;
  long long cap = resident_blocks(kernel, kUpdateThreads, lds);
  if (cap > kMaxBlocks) cap = kMaxBlocks;
  if (cap < 1) cap = 1;
  // every block strides over the same number of tiles (no half-empty round)
  const long long rounds = (tiles + cap - 1) / cap;
  long long g = (tiles + rounds - 1) / rounds;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
using UpdateKernel = void (*)(Work, long long, int, int, T*, long long, const T*, const double*,
                              const double*, double, int);

// Row vectors per thread of the single-instance update: the largest of 8
// (FP64 only: the FP32 accumulators would not leave two blocks per CU), 4, 2
// and 1 whose tiles still number at least one per CU; 0 (the column split)
// when the solve allows it and even one vector per thread gives fewer tiles
// than half the CUs.
template <typename T>
static int update_nv(long long n, bool col_split) {
  const long long cus = resident_blocks(nullptr, 0, 0);
  if (sizeof(T) == 8 && (n + update_tile_rows<T, 8>() - 1) / update_tile_rows<T, 8>() >= cus)
    return 8;
  if ((n + update_tile_rows<T, 4>() - 1) / update_tile_rows<T, 4>() >= cus) return 4;
  if ((n + update_tile_rows<T, 2>() - 1) / update_tile_rows<T, 2>() >= cus) return 2;
  if (!col_split || (n + update_tile_rows<T, 1>() - 1) / update_tile_rows<T, 1>() >= cus / 2)
    return 1;
  return 0;
}

template <typename T>
static hipError_t update_dispatch(const Work& w, long long n, int j, bool has_t, int ngroups,
                                  T* Vraw, long long ldv_raw, const T* zraw, const double* traw,
                                  const double* r1raw, double igraw, int raw, hipStream_t s) {
  // 16-byte row vectors need a leading dimension of whole vectors and
  // 16-byte aligned columns
  const T* Vp = (raw == 1) ? Vraw : basis<T>(w);
  const T* zp = (raw == 1) ? zraw : zvec<T>(w);
  const long long ldv = (raw == 1) ? ldv_raw : w.ldv;
  const bool vec = (ldv % Vec16<T>::W == 0) && (reinterpret_cast<uintptr_t>(Vp) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(zp) % 16 == 0);
  // the longest runs per column that still give every CU a tile
  const int nv = vec ? update_nv<T>(n, raw == 0 && w.col_split) : 2;
  UpdateKernel<T> k;
  long long tile_rows;
  if (nv == 8) {
    k = has_t ? update_kernel<true, true, T, 8> : update_kernel<false, true, T, 8>;
    tile_rows = update_tile_rows<T, 8>();
  } else if (nv == 4) {
    k = has_t ? update_kernel<true, true, T, 4> : update_kernel<false, true, T, 4>;
    tile_rows = update_tile_rows<T, 4>();
  } else if (nv == 1) {
    k = has_t ? update_kernel<true, true, T, 1> : update_kernel<false, true, T, 1>;
    tile_rows = update_tile_rows<T, 1>();
  } else if (nv == 0) {
    k = has_t ? update_kernel<true, true, T, 0> : update_kernel<false, true, T, 0>;
    tile_rows = (long long)kWave * Vec16<T>::W;
  } else {
    k = has_t ? (vec ? update_kernel<true, true, T, 2> : update_kernel<true, false, T, 2>)
              : (vec ? update_kernel<false, true, T, 2> : update_kernel<false, false, T, 2>);
    tile_rows = update_tile_rows<T, 2>();
  }
  const size_t lds = update_lds_doubles(j) * sizeof(double);
  unsigned grid = update_grid(reinterpret_cast<const void*>(k), n, tile_rows, lds);
  if (raw == 0 && w.tune && (w.tune[j] & 2) && grid > 1) grid = (grid + 1) / 2;
  Work wa = w;
  long long na = n, ldva = ldv_raw;
  int ja = j, nga = ngroups, rawa = raw;
  T* va = Vraw;
  const T* za = zraw;
  const double* ta = traw;
  const double* ra = r1raw;
  double iga = igraw;
  void* args[] = {&wa, &na, &ja, &nga, &va, &ldva, &za, &ta, &ra, &iga, &rawa};
  return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(grid), dim3(kUpdateThreads), args,
                         lds, s);
}

hipError_t launch_update(const Work& w, long long n, int j, int gs, int ngroups, hipStream_t s) {
  // With one Gauss-Seidel sweep there is no second-sweep vector t, and the
  // kernel variant without it skips one FMA stream.
  if (w.fp32)
    return update_dispatch<float>(w, n, j, gs == 2, ngroups, nullptr, 0, nullptr, nullptr,
                                  nullptr, 0.0, 0, s);
  return update_dispatch<double>(w, n, j, gs == 2, ngroups, nullptr, 0, nullptr, nullptr, nullptr,
                                 0.0, 0, s);
}

hipError_t launch_correct(const Work& w, long long n, int j, int ngroups, hipStream_t s) {
  if (w.fp32)
    return update_dispatch<float>(w, n, j, true, ngroups, nullptr, 0, nullptr, nullptr, nullptr,
                                  1.0, 2, s);
  return update_dispatch<double>(w, n, j, true, ngroups, nullptr, 0, nullptr, nullptr, nullptr,
                                 1.0, 2, s);
}

hipError_t launch_update_raw(double* V, long long ldv, long long n, int j, const double* z,
                             const double* t, const double* r1, double inv_gamma, hipStream_t s) {
  Work w{};
  return update_dispatch<double>(w, n, j, true, 0, V, ldv, z, t, r1, inv_gamma, 1, s);
}

// ---------------------------------------------------------------------------
// End of cycle: R y = g by back substitution (one block), then x += V y
// ---------------------------------------------------------------------------

// Panel width so that the right-hand side plus one panel of R stay within
// 64 KiB of shared memory.
static int lsq_panel(int m) {
  if (m < 1) m = 1;
  int p = (8000 - m) / m;
  if (p > 32) p = 32;
  if (p < 1) p = 1;
  return p;
}

__device__ __forceinline__ void lsq_body(const Work& w, int panel) {
  extern __shared__ double sm[];
  const int J = load_agent(&w.ctl->J);
  if (J <= 0) return;
  double* sb = sm;               // right-hand side, updated in place
  double* sp = sm + J + 1;       // panel of R: rows 0..hi-1, `panel` columns
  for (int i = threadIdx.x; i < J; i += blockDim.x) sb[i] = w.g[i];
  for (int hi = J; hi > 0; hi -= panel) {
    const int lo = hi > panel ? hi - panel : 0;
    const int pw = hi - lo;
    __syncthreads();
    for (int idx = threadIdx.x; idx < pw * hi; idx += blockDim.x) {
      const int c = idx / hi;
      const int i = idx % hi;
      sp[(size_t)c * hi + i] = w.R[(size_t)(lo + c) * w.ldh + i];
    }
    __syncthreads();
    for (int c = hi - 1; c >= lo; --c) {
      const double* col = sp + (size_t)(c - lo) * hi;
      const double yc = sb[c] / col[c];
      __syncthreads();
      for (int i = threadIdx.x; i < c; i += blockDim.x) sb[i] = fma(-col[i], yc, sb[i]);
      if (threadIdx.x == 0) {
        w.y[c] = yc;
        sb[c] = yc;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void lsq_kernel(Work w, int panel) { lsq_body(w, panel); }

hipError_t launch_lsq(const Work& w, int m, hipStream_t s) {
  const int panel = lsq_panel(m);
  const size_t lds = ((size_t)m + 1 + (size_t)panel * m) * sizeof(double);
  hipLaunchKernelGGL(lsq_kernel, dim3(1), dim3(256), lds, s, w, panel);
  return hipGetLastError();
}

// x += V_{0:J} y (x and y FP64; V in the basis element type T), each row's
// products added in column order and then to x.  NV > 0: tiles of NV
// 16-byte row vectors per thread (runs of NV x 4 KB per column and block, as
// the update takes them), the column loads in two alternating register
// stages; rows past the last whole tile, or arrays the vectors cannot take,
// one row per thread.  NV = 0: tiles of kUpdateRows rows per thread, element
// loads.
template <typename T, int NV>
__device__ __forceinline__ void xupdate_vec(Grid gr, const Work& w, long long n,
                                            double* __restrict__ x, int J) {
  typedef typename Vec16<T>::type VT;
  constexpr int W = Vec16<T>::W;
  constexpr long long kTile = (long long)NV * W * kUpdateThreads;
  const double* __restrict__ y = w.y;
  const T* __restrict__ V = basis<T>(w);
  const long long ntiles = (n + kTile - 1) / kTile;
  for (long long tile = gr.bid; tile < ntiles; tile += gr.nb) {
    const long long tb = tile * kTile;
    if (tb + kTile <= n) {
      long long p[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k)
        p[k] = tb + (long long)W * threadIdx.x + (long long)k * W * kUpdateThreads;
      double acc[NV][W];
#pragma unroll
      for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int e = 0; e < W; ++e) acc[k][e] = 0.0;
      auto load = [&](VT* v, int c) {
        const T* vc = V + (size_t)c * w.ldv;
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = ld16_stream<T>(vc + p[k]);
      };
      auto use = [&](const VT* v, int c) {
        const double yc = y[c];
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
          for (int e = 0; e < W; ++e) acc[k][e] = fma((double)v[k][e], yc, acc[k][e]);
      };
      VT va[NV], vb[NV];
      int c = 0;
      load(va, 0);
      while (true) {
        load(vb, (c + 1 < J) ? c + 1 : c);
        use(va, c);
        if (++c >= J) break;
        load(va, (c + 1 < J) ? c + 1 : c);
        use(vb, c);
        if (++c >= J) break;
      }
#pragma unroll
      for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int h = 0; h < W; h += 2) {
          double2 xv = *reinterpret_cast<const double2*>(x + p[k] + h);
          xv.x += acc[k][h];
          xv.y += acc[k][h + 1];
          *reinterpret_cast<double2*>(x + p[k] + h) = xv;
        }
      continue;
    }
    // the ragged last tile: one row per thread
    const long long te = min(n, tb + kTile);
    for (long long r = tb + threadIdx.x; r < te; r += kUpdateThreads) {
      double acc = 0.0;
      for (int c = 0; c < J; ++c) acc = fma((double)V[(size_t)c * w.ldv + r], y[c], acc);
      x[r] += acc;
    }
  }
}

template <typename T, int NV>
__device__ __forceinline__ void xupdate_body(Grid gr, const Work& w, long long n,
                                             double* __restrict__ x) {
  const int J = load_agent(&w.ctl->J);
  if (J <= 0) return;
  if constexpr (NV > 0) {
    const bool vec = (w.ldv % Vec16<T>::W == 0) &&
                     (reinterpret_cast<uintptr_t>(basis<T>(w)) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(x) % 16 == 0);
    if (vec) {
      xupdate_vec<T, NV>(gr, w, n, x, J);
      return;
    }
  }
  const double* __restrict__ y = w.y;
  const T* __restrict__ V = basis<T>(w);
  constexpr long long kTile = (long long)kUpdateThreads * kUpdateRows;
  const long long ntiles = (n + kTile - 1) / kTile;
  for (long long tile = gr.bid; tile < ntiles; tile += gr.nb) {
    const long long base = tile * kTile + threadIdx.x;
    double acc[kUpdateRows];
#pragma unroll
    for (int k = 0; k < kUpdateRows; ++k) acc[k] = 0.0;
    const bool full = base + (long long)(kUpdateRows - 1) * kUpdateThreads < n;
    int c = 0;
    if (full) {
      for (; c + 4 <= J; c += 4) {
        double vv[4][kUpdateRows];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const T* __restrict__ vc = V + (size_t)(c + cc) * w.ldv + base;
#pragma unroll
          for (int k = 0; k < kUpdateRows; ++k) vv[cc][k] = (double)vc[k * kUpdateThreads];
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const double yc = y[c + cc];
#pragma unroll
          for (int k = 0; k < kUpdateRows; ++k) acc[k] = fma(vv[cc][k], yc, acc[k]);
        }
      }
    }
    for (; c < J; ++c) {
      const T* __restrict__ vc = V + (size_t)c * w.ldv + base;
      const double yc = y[c];
#pragma unroll
      for (int k = 0; k < kUpdateRows; ++k) {
        if (base + k * kUpdateThreads < n) acc[k] = fma((double)vc[k * kUpdateThreads], yc, acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kUpdateRows; ++k) {
      const long long r = base + k * kUpdateThreads;
      if (r < n) x[r] += acc[k];
    }
  }
}

template <typename T, int NV>
__global__ __launch_bounds__(kUpdateThreads) void xupdate_kernel(Work w, long long n,
                                                                double* __restrict__ x) {
  xupdate_body<T, NV>(hw_grid(), w, n, x);
}

// One tile per block: eight row vectors of doubles (four of floats) per
// thread when that still gives every CU a tile, else four, else element
// loads with kUpdateRows rows per thread.
template <typename T>
static hipError_t xupdate_dispatch(const Work& w, long long n, double* x, hipStream_t s) {
  const long long cus = resident_blocks(nullptr, 0, 0);
  constexpr int W = Vec16<T>::W;
  const long long t8 = (n + 8LL * W * kUpdateThreads - 1) / (8LL * W * kUpdateThreads);
  const long long t4 = (n + 4LL * W * kUpdateThreads - 1) / (4LL * W * kUpdateThreads);
  const void* k;
  long long g;
  if (sizeof(T) == 8 && t8 >= cus) {
    k = reinterpret_cast<const void*>(xupdate_kernel<T, 8>);
    g = t8;
  } else if (t4 >= cus) {
    k = reinterpret_cast<const void*>(xupdate_kernel<T, 4>);
    g = t4;
  } else {
    const long long per = (long long)kUpdateThreads * kUpdateRows;
    k = reinterpret_cast<const void*>(xupdate_kernel<T, 0>);
    g = (n + per - 1) / per;
  }
  if (g > kMaxBlocks) g = kMaxBlocks;
  Work wa = w;
  long long na = n;
  double* xa = x;
  void* args[] = {&wa, &na, &xa};
  return hipLaunchKernel(k, dim3((unsigned)g), dim3(kUpdateThreads), args, 0, s);
}

hipError_t launch_xupdate(const Work& w, long long n, double* x, hipStream_t s) {
  if (w.fp32) return xupdate_dispatch<float>(w, n, x, s);
  return xupdate_dispatch<double>(w, n, x, s);
}

// ---------------------------------------------------------------------------
// Comparator: modified Gram-Schmidt Arnoldi (the textbook GMRES the paper
// measures IGS-GMRES against), FP64.  Column c takes w = A v_c in V[:, c+1],
// then c + 2 kernels, each one grid-wide reduction: kernel i applies the
// previous projection w -= H[i-1, c] v_{i-1} and forms H[i, c] = v_i^T w
// (i <= c) or ||w||^2 (i = c + 1, whose last block finishes the column: the
// Givens rotation, the breakdown and stopping tests), then v_{c+1} = w / H[c+1, c].
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kUpdateThreads) void mgs_kernel(Work w, long long n, int c, int i) {
  __shared__ double red[kUpdateThreads / kWave];
  __shared__ double tot[1];
  __shared__ double scr[kUpdateThreads];
  __shared__ double hcol[kMgsMaxCols + 2];
  if (!ctl_runs(w.ctl, c)) return;
  const Grid gr = hw_grid();
  double* __restrict__ wv = w.V + (size_t)(c + 1) * w.ldv;
  double* hc = w.H + hess_col(c);
  const double hp = (i > 0) ? hc[i - 1] : 0.0;
  const double* __restrict__ vp = w.V + (size_t)(i > 0 ? i - 1 : 0) * w.ldv;
  const double* __restrict__ vi = w.V + (size_t)(i <= c ? i : 0) * w.ldv;
  constexpr long long kTile = (long long)kUpdateThreads * kUpdateRows;
  const long long ntiles = (n + kTile - 1) / kTile;
  double acc = 0.0;
  for (long long tile = gr.bid; tile < ntiles; tile += gr.nb) {
#pragma unroll
    for (int k = 0; k < kUpdateRows; ++k) {
      const long long r = tile * kTile + (long long)k * kUpdateThreads + threadIdx.x;
      if (r < n) {
        double x = wv[r];
        if (i > 0) x = fma(-hp, vp[r], x);
        wv[r] = x;
        acc = fma((i <= c) ? vi[r] : x, x, acc);
      }
    }
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < kUpdateThreads / kWave; ++k) a += red[k];
    put_partial(w.part + (size_t)gr.bid * w.pstride, a);
  }
  if (!grid_reduce_last(w.part, w.gpart, w.pstride, w.tickets, 1, tot, scr, gr)) return;
  const double total = tot[0];
  if (i <= c) {
    if (threadIdx.x == 0) hc[i] = total;
    return;
  }
  // last block of the last kernel of column c: finish it
  Ctl* ctl = w.ctl;
  if (!isfinite(total)) {
    if (threadIdx.x == 0) {
      ctl->status = kNonfinite;
      ctl->J = c;
      ctl->end_iter = c;
    }
    return;
  }
  const double gamma = sqrt(total);
  for (int q = threadIdx.x; q <= c; q += blockDim.x) hcol[q] = hc[q];
  __shared__ double s_gc;
  if (threadIdx.x == 0) s_gc = w.g[c];
  __syncthreads();
  const int brk = finish_column(w, c + 1, hcol, gamma, w.cs, w.sn, s_gc, n);
  if (threadIdx.x == 0) {
    int code = kRunning;
    if (brk) code = kBreakdown;
    else if (ctl->gabs <= ctl->tol_cyc) code = kConverged;
    else if (c + 1 >= ctl->m) code = kFull;
    else if (ctl->its_before + c + 1 >= ctl->maxit) code = kMaxit;
    if (code != kRunning) {
      ctl->status = code;
      ctl->J = c + 1;
      ctl->end_iter = c;
      if (brk) ctl->breakdowns += 1;
    }
  }
}

// ||r0|| at the start of an MGS cycle (r0 in V[:, 0]); the last block sets
// rho and g[0] and ends the cycle at once when it has converged or the
// iteration budget is used up.
__global__ __launch_bounds__(kUpdateThreads) void mgs_norm0_kernel(Work w, long long n) {
  __shared__ double red[kUpdateThreads / kWave];
  __shared__ double tot[1];
  __shared__ double scr[kUpdateThreads];
  const Grid gr = hw_grid();
  const double* __restrict__ v = w.V;
  constexpr long long kTile = (long long)kUpdateThreads * kUpdateRows;
  const long long ntiles = (n + kTile - 1) / kTile;
  double acc = 0.0;
  for (long long tile = gr.bid; tile < ntiles; tile += gr.nb) {
#pragma unroll
    for (int k = 0; k < kUpdateRows; ++k) {
      const long long r = tile * kTile + (long long)k * kUpdateThreads + threadIdx.x;
      if (r < n) acc = fma(v[r], v[r], acc);
    }
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < kUpdateThreads / kWave; ++k) a += red[k];
    put_partial(w.part + (size_t)gr.bid * w.pstride, a);
  }
  if (!grid_reduce_last(w.part, w.gpart, w.pstride, w.tickets, 1, tot, scr, gr)) return;
  if (threadIdx.x != 0) return;
  Ctl* ctl = w.ctl;
  const double rho = sqrt(tot[0]);
  ctl->rho = rho;
  ctl->gabs = rho;
  w.g[0] = rho;
  if (!isfinite(rho)) {
    ctl->status = kNonfinite;
    ctl->J = 0;
    ctl->end_iter = -1;
  } else if (rho <= ctl->tol_abs || ctl->its_before >= ctl->maxit) {
    ctl->status = (rho <= ctl->tol_abs) ? kConvStart : kMaxit;
    ctl->J = 0;
    ctl->end_iter = -1;
  }
}

// V[:, col] /= *d while iteration gate_j runs and *d > 0.
__global__ __launch_bounds__(kUpdateThreads) void mgs_scale_kernel(Work w, long long n, int col,
                                                                 const double* d, int gate_j) {
  if (!ctl_runs(w.ctl, gate_j)) return;
  const double g = *d;
  if (!(g > 0.0)) return;
  double* __restrict__ v = w.V + (size_t)col * w.ldv;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x)
    v[r] = v[r] / g;
}

static unsigned mgs_grid(long long n) {
  const long long per = (long long)kUpdateThreads * kUpdateRows;
  long long g = (n + per - 1) / per;
  const long long cap = resident_blocks(reinterpret_cast<const void*>(mgs_kernel), kUpdateThreads, 0);
  if (g > cap) g = cap;
  if (g > kMaxBlocks) g = kMaxBlocks;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_mgs_start(const Work& w, long long n, hipStream_t s) {
  const unsigned g = mgs_grid(n);
  hipLaunchKernelGGL(mgs_norm0_kernel, dim3(g), dim3(kUpdateThreads), 0, s, w, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mgs_scale_kernel, dim3(g), dim3(kUpdateThreads), 0, s, w, n, 0,
                     reinterpret_cast<const double*>(&w.ctl->rho), 0);
  return hipGetLastError();
}

hipError_t launch_mgs_column(const Work& w, long long n, int c, hipStream_t s) {
  if (c + 1 > kMgsMaxCols) return hipErrorInvalidValue;
  const unsigned g = mgs_grid(n);
  for (int i = 0; i <= c + 1; ++i) {
    hipLaunchKernelGGL(mgs_kernel, dim3(g), dim3(kUpdateThreads), 0, s, w, n, c, i);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(mgs_scale_kernel, dim3(g), dim3(kUpdateThreads), 0, s, w, n, c + 1,
                     reinterpret_cast<const double*>(w.H + hess_col(c) + c + 1), c);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batches: one launch runs the same step for many independent instances
// ---------------------------------------------------------------------------

// Instance k of a launch owns blocks [start, start + nblk) of the grid
// (start a multiple of 8); aux carries a per-instance launch parameter.
struct MapEntry {
  int start;
  int nblk;
  int inst;
  int pad;
  long long aux;
};
struct BatchMap {
  int count;
  int total;
  MapEntry e[kMaxBatch];
};

// The entry that owns this block: a scan over compile-time indices of the
// kernel argument (no dynamic indexing into it).
__device__ __forceinline__ MapEntry map_find(const BatchMap& m) {
  MapEntry r = m.e[0];
#pragma unroll
  for (int k = 1; k < kMaxBatch; ++k)
    if (k < m.count && (int)blockIdx.x >= m.e[k].start) r = m.e[k];
  return r;
}

template <int LPR, int RPG, typename T, bool RESID>
__global__ __launch_bounds__(256) void spmv_batch_kernel(const Inst* __restrict__ tab,
                                                         BatchMap map, int j) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const Inst I = tab[e.inst];
  const Grid gr{bid, e.nblk};
  if constexpr (RESID) {
    // r = b - A x in FP64, stored in the basis element type
    spmv_csr_body<LPR, RPG, double, T>(gr, I.n, I.op.row_ptr, I.op.col_idx, I.op.vals, I.x,
                                       basis<T>(I.w), I.b, nullptr, 0);
  } else {
    spmv_csr_body<LPR, RPG, T, T>(gr, I.n, I.op.row_ptr, I.op.col_idx, op_vals<T>(I.op),
                                  basis<T>(I.w) + (size_t)j * I.w.ldv, zvec<T>(I.w), nullptr,
                                  I.w.ctl, j);
  }
}

template <int CPW, bool VEC, bool Z, typename T>
__global__ __launch_bounds__(kReduceThreads) void reduce_batch_kernel(const Inst* __restrict__ tab,
                                                                      BatchMap map, int j, int cpw,
                                                                      int wc, int wr) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  // copies taken before any store, so that they load through the scalar
  // path and live in scalar registers as kernel arguments would
  const Work w = tab[e.inst].w;
  const long long n = tab[e.inst].n;
  reduce_body<CPW, VEC, Z, T>(Grid{bid, e.nblk}, w, n, j, e.aux, cpw, wc, wr, nullptr, 0, nullptr,
                              nullptr);
}

// Row vectors per thread of the batched update (tiles of 2,048 FP64 rows):
// 16 KB runs per column, as the single-instance update takes on large n.
constexpr int kBatchNV = 4;

template <bool HAS_T, bool VEC, typename T>
__global__ __launch_bounds__(kUpdateThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 1))) void update_batch_kernel(
    const Inst* __restrict__ tab, BatchMap map, int j) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const Work w = tab[e.inst].w;
  const long long n = tab[e.inst].n;
  update_body<HAS_T, VEC, T, kBatchNV>(Grid{bid, e.nblk}, w, n, j, (int)e.aux, nullptr, 0,
                                       nullptr, nullptr, nullptr, 0.0, 0);
}

__global__ __launch_bounds__(256) void bnorm_batch_kernel(const Inst* __restrict__ tab,
                                                          BatchMap map) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const Inst I = tab[e.inst];
  bnorm_body(Grid{bid, e.nblk}, I.b, I.x, I.n, I.w);
}

__global__ void cycle_begin_batch_kernel(const Inst* __restrict__ tab, BatchMap map) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk || threadIdx.x != 0) return;
  const Inst& I = tab[e.inst];
  cycle_begin_body(I.w.ctl, I.its_before, I.maxit, I.m, I.gs, I.final_v, I.tol, I.tau,
                   I.cycle_rtol);
}

__global__ __launch_bounds__(256) void lsq_batch_kernel(const Inst* __restrict__ tab, BatchMap map,
                                                        int panel) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const Work w = tab[e.inst].w;
  if (!tab[e.inst].run_lsq) return;
  lsq_body(w, panel);
}

template <typename T>
__global__ __launch_bounds__(kUpdateThreads) void xupdate_batch_kernel(const Inst* __restrict__ tab,
                                                                       BatchMap map) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const Inst I = tab[e.inst];
  if (!I.run_lsq) return;
  xupdate_body<T, 0>(Grid{bid, e.nblk}, I.w, I.n, I.x);
}

__global__ void ctl_gather_kernel(const Inst* __restrict__ tab, BatchMap map, Ctl* out) {
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const int* src = reinterpret_cast<const int*>(tab[e.inst].w.ctl);
  int* dst = reinterpret_cast<int*>(out + e.inst);
  for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int)); i += blockDim.x) dst[i] = src[i];
}

// Lay out the instances act[k] of a launch with nblk[k] blocks each.
static void build_map(BatchMap& m, const BatchRun& r, const int* nblk, const long long* aux) {
  m.count = r.count;
  int start = 0;
  for (int k = 0; k < r.count; ++k) {
    m.e[k] = MapEntry{start, nblk[k], r.act[k], 0, aux ? aux[k] : 0};
    start += (nblk[k] + 7) / 8 * 8;
  }
  for (int k = r.count; k < kMaxBatch; ++k) m.e[k] = MapEntry{start, 0, 0, 0, 0};
  m.total = start;
}

static bool batch_fp32(const BatchRun& r) { return r.h_tab[r.act[0]].w.fp32 != 0; }

// 16-byte row vectors for every instance (whole vectors per column, aligned
// columns); the batch kernels have no element path for other layouts.
template <typename T>
static bool batch_vec(const BatchRun& r) {
  for (int k = 0; k < r.count; ++k) {
    const Work& w = r.h_tab[r.act[k]].w;
    if (w.ldv % Vec16<T>::W != 0 || reinterpret_cast<uintptr_t>(basis<T>(w)) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(zvec<T>(w)) % 16 != 0)
      return false;
  }
  return true;
}

static hipError_t launch_map(const void* kernel, const BatchMap& m, unsigned threads, size_t lds,
                             void** args, hipStream_t s) {
  if (m.total == 0) return hipSuccess;
  return hipLaunchKernel(kernel, dim3((unsigned)m.total), dim3(threads), args, lds, s);
}

hipError_t batch_bnorm(const BatchRun& r) {
  if (r.count <= 0) return hipSuccess;
  int nb[kMaxBatch];
  for (int k = 0; k < r.count; ++k) {
    long long blocks = (r.h_tab[r.act[k]].n + 255) / 256;   // as launch_bnorm
    nb[k] = (int)(blocks > 1024 ? 1024 : blocks);
  }
  BatchMap m;
  build_map(m, r, nb, nullptr);
  const Inst* t = r.d_tab;
  void* args[] = {&t, &m};
  return launch_map(reinterpret_cast<const void*>(bnorm_batch_kernel), m, 256, 0, args, r.stream);
}

// The operator apply of the instances that hold an ELL form, RPT rows per
// thread: the products and additions of spmv_ell_kernel (and so of the
// CSR kernel with 8 lanes per row), with the slot count K read from the
// instance; so z is bit-identical to a lone solve's.
template <int RPT, typename T>
__global__ __launch_bounds__(256) void spmv_ell_batch_kernel(const Inst* __restrict__ tab,
                                                             BatchMap map, int j) {
#pragma clang fp contract(off)
  typedef int IV __attribute__((ext_vector_type(RPT)));
  typedef T AV __attribute__((ext_vector_type(RPT)));
  const MapEntry e = map_find(map);
  const int bid = (int)blockIdx.x - e.start;
  if (bid >= e.nblk) return;
  const Inst* I = tab + e.inst;
  const Work w = I->w;
  if (!ctl_runs(w.ctl, j)) return;
  const long long n = I->n;
  const long long row0 = ((long long)bid * blockDim.x + threadIdx.x) * RPT;
  if (row0 >= n) return;
  const int K = I->op.ell_k;
  const int* __restrict__ col = I->op.ell_col;
  const T* __restrict__ val = ell_vals<T>(I->op);
  const T* __restrict__ x = basis<T>(w) + (size_t)j * w.ldv;
  T* __restrict__ y = zvec<T>(w);
  IV c[8];
  AV v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < K) {
      c[k] = *reinterpret_cast<const IV*>(col + (long long)k * n + row0);
      v[k] = *reinterpret_cast<const AV*>(val + (long long)k * n + row0);
    } else {
      c[k] = IV(0);
      v[k] = AV(0);
    }
  }
  AV out;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    T p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = v[k][i] * x[c[k][i]];
    const T q0 = (p[0] + p[1]) + (p[2] + p[3]);
    const T q1 = (p[4] + p[5]) + (p[6] + p[7]);
    out[i] = q0 + q1;
  }
  __builtin_nontemporal_store(out, reinterpret_cast<AV*>(y + row0));   // see st16
}

// The instances of r with an ELL form (and no tuned CSR shape): one launch
// for those with even n (two rows per thread), one for the others.
template <typename T>
static hipError_t batch_spmv_ell(const BatchRun& r, int j) {
  for (int rpt = 2; rpt >= 1; --rpt) {
    BatchRun sub = r;
    sub.count = 0;
    int nb[kMaxBatch];
    for (int q = 0; q < r.count; ++q) {
      const Inst& I = r.h_tab[r.act[q]];
      const int want = (I.n % 2 == 0) ? 2 : 1;
      if (want != rpt) continue;
      nb[sub.count] = (int)((I.n / rpt + 255) / 256);
      sub.act[sub.count++] = r.act[q];
    }
    if (sub.count == 0) continue;
    BatchMap m;
    build_map(m, sub, nb, nullptr);
    const Inst* t = r.d_tab;
    int ja = j;
    void* args[] = {&t, &m, &ja};
    const void* kern = (rpt == 2) ? reinterpret_cast<const void*>(spmv_ell_batch_kernel<2, T>)
                                  : reinterpret_cast<const void*>(spmv_ell_batch_kernel<1, T>);
    const hipError_t err = launch_map(kern, m, 256, 0, args, r.stream);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

static bool inst_has_ell(const Inst& I) {
  return I.op.ell_k > 0 && I.op.rpg == 0 && I.op.ell_col != nullptr &&
         (I.w.fp32 ? I.op.ell_val32 != nullptr : I.op.ell_val != nullptr);
}

// The operator apply for the instances with lanes-per-row `lpr` (one launch
// per distinct value; RESID: the residual r = b - A x of the cycle start).
template <typename T, bool RESID>
static hipError_t batch_spmv_lpr(const BatchRun& r, int j) {
  bool seen[7] = {false, false, false, false, false, false, false};
  for (int k = 0; k < r.count; ++k) {
    const int lpr = r.h_tab[r.act[k]].op.lpr;
    int li = 0;
    while ((1 << li) < lpr) ++li;
    if ((1 << li) != lpr || li > 6) return hipErrorInvalidValue;
    if (seen[li]) continue;
    seen[li] = true;
    BatchRun sub = r;
    sub.count = 0;
    int nb[kMaxBatch];
    for (int q = 0; q < r.count; ++q) {
      const Inst& I = r.h_tab[r.act[q]];
      if (I.op.lpr != lpr) continue;
      nb[sub.count] = (int)spmv_grid(I.n, lpr, spmv_rpg(lpr));
      sub.act[sub.count++] = r.act[q];
    }
    BatchMap m;
    build_map(m, sub, nb, nullptr);
    const Inst* t = r.d_tab;
    int ja = j;
    void* args[] = {&t, &m, &ja};
    const void* kern = nullptr;
    switch (lpr) {
#define IGS_BSPMV_CASE(L, R) \
  case L: kern = reinterpret_cast<const void*>(spmv_batch_kernel<L, R, T, RESID>); break;
      IGS_BSPMV_CASE(1, LPR_RPG_MAX) IGS_BSPMV_CASE(2, LPR_RPG_MAX) IGS_BSPMV_CASE(4, LPR_RPG_MAX)
      IGS_BSPMV_CASE(8, LPR_RPG_MAX) IGS_BSPMV_CASE(16, 2) IGS_BSPMV_CASE(32, 1)
      IGS_BSPMV_CASE(64, 1)
#undef IGS_BSPMV_CASE
      default: return hipErrorInvalidValue;
    }
    const hipError_t err = launch_map(kern, m, 256, 0, args, r.stream);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t batch_residual(const BatchRun& r) {
  if (r.count <= 0) return hipSuccess;
  int nb[kMaxBatch];
  for (int k = 0; k < r.count; ++k) nb[k] = 1;
  BatchMap m;
  build_map(m, r, nb, nullptr);
  const Inst* t = r.d_tab;
  void* args[] = {&t, &m};
  hipError_t e =
      launch_map(reinterpret_cast<const void*>(cycle_begin_batch_kernel), m, 64, 0, args, r.stream);
  if (e != hipSuccess) return e;
  return batch_fp32(r) ? batch_spmv_lpr<float, true>(r, 0) : batch_spmv_lpr<double, true>(r, 0);
}

hipError_t batch_spmv(const BatchRun& r, int j) {
  if (r.count <= 0) return hipSuccess;
  // members with an ELL form take the ELL kernel, the others the CSR one
  BatchRun ell = r, csr = r;
  ell.count = csr.count = 0;
  for (int q = 0; q < r.count; ++q) {
    if (inst_has_ell(r.h_tab[r.act[q]])) ell.act[ell.count++] = r.act[q];
    else csr.act[csr.count++] = r.act[q];
  }
  const bool f32 = batch_fp32(r);
  if (ell.count > 0) {
    const hipError_t e = f32 ? batch_spmv_ell<float>(ell, j) : batch_spmv_ell<double>(ell, j);
    if (e != hipSuccess) return e;
  }
  if (csr.count == 0) return hipSuccess;
  return f32 ? batch_spmv_lpr<float, false>(csr, j) : batch_spmv_lpr<double, false>(csr, j);
}

template <typename T>
static const void* pick_reduce_batch(int tcpw, bool z) {
  switch (tcpw * 2 + (z ? 1 : 0)) {
#define IGS_BRED_CASE(C, ZZ) \
  case C * 2 + ZZ: return reinterpret_cast<const void*>(reduce_batch_kernel<C, true, ZZ, T>);
    IGS_BRED_CASE(1, 0) IGS_BRED_CASE(1, 1) IGS_BRED_CASE(2, 0) IGS_BRED_CASE(2, 1)
    IGS_BRED_CASE(4, 0) IGS_BRED_CASE(4, 1) IGS_BRED_CASE(8, 0) IGS_BRED_CASE(8, 1)
#undef IGS_BRED_CASE
    default: return nullptr;
  }
}

template <typename T>
static hipError_t batch_reduce_t(const BatchRun& r, int j, bool with_z, int* ngroups) {
  const int ncol = j + 1;
  const ReduceShape sh0 = reduce_shape(j);
  const size_t lds = reduce_lds_bytes(sh0, ncol);
  if (!batch_vec<T>(r)) return hipErrorInvalidValue;
  const void* kern = pick_reduce_batch<T>(sh0.tcpw, with_z);
  if (kern == nullptr) return hipErrorInvalidValue;
  // each instance's grid is the one reduce_dispatch launches for it alone
  int cap = resident_blocks(reinterpret_cast<const void*>(pick_reduce<T>(sh0.tcpw, true, true)),
                            kReduceThreads, lds);
  if (cap > kMaxBlocks) cap = kMaxBlocks;
  if (sh0.tcpw <= 2) {
    const int cus = resident_blocks(nullptr, 0, 0);
    if (cap > cus) cap = cus;
  }
  int nb[kMaxBatch];
  long long rpb[kMaxBatch];
  const long long rmin = r.reduce_rows > 1 ? r.reduce_rows : 1;
  for (int k = 0; k < r.count; ++k) {
    ReduceShape sh = sh0;
    // an instance's grid depends on its own n and j only, never on the
    // other members of the launch
    const long long n = r.h_tab[r.act[k]].n;
    const long long want = (n + rmin - 1) / rmin;
    reduce_rows(sh, n, (int)(want < cap ? want : cap));
    nb[k] = sh.nblocks;
    rpb[k] = sh.rows_per_block;
    ngroups[k] = reduce_groups(sh.nblocks);
  }
  BatchMap m;
  build_map(m, r, nb, rpb);
  const Inst* t = r.d_tab;
  int ja = j, cpw = sh0.cpw, wc = sh0.wc, wr = sh0.wr;
  void* args[] = {&t, &m, &ja, &cpw, &wc, &wr};
  return launch_map(kern, m, kReduceThreads, lds, args, r.stream);
}

hipError_t batch_reduce(const BatchRun& r, int j, bool with_z, int* ngroups) {
  if (r.count <= 0) return hipSuccess;
  return batch_fp32(r) ? batch_reduce_t<float>(r, j, with_z, ngroups)
                       : batch_reduce_t<double>(r, j, with_z, ngroups);
}

template <typename T>
static hipError_t batch_update_t(const BatchRun& r, int j, const int* ngroups) {
  if (!batch_vec<T>(r)) return hipErrorInvalidValue;
  const bool has_t = r.h_tab[r.act[0]].gs == 2;
  const void* kern = has_t ? reinterpret_cast<const void*>(update_batch_kernel<true, true, T>)
                           : reinterpret_cast<const void*>(update_batch_kernel<false, true, T>);
  const void* lone = has_t ? reinterpret_cast<const void*>(update_kernel<true, true, T, kBatchNV>)
                           : reinterpret_cast<const void*>(update_kernel<false, true, T, kBatchNV>);
  const size_t lds = update_lds_doubles(j) * sizeof(double);
  int nb[kMaxBatch];
  long long ng[kMaxBatch];
  const long long tmin = r.update_tiles > 1 ? r.update_tiles : 1;
  for (int k = 0; k < r.count; ++k) {
    const long long n = r.h_tab[r.act[k]].n;
    constexpr long long kRows = update_tile_rows<T, kBatchNV>();
    const long long g = update_grid(lone, n, kRows, lds);
    const long long tiles = (n + kRows - 1) / kRows;
    const long long want = (tiles + tmin - 1) / tmin;
    nb[k] = (int)(want < g ? want : g);
    ng[k] = ngroups[k];
  }
  BatchMap m;
  build_map(m, r, nb, ng);
  const Inst* t = r.d_tab;
  int ja = j;
  void* args[] = {&t, &m, &ja};
  return launch_map(kern, m, kUpdateThreads, lds, args, r.stream);
}

hipError_t batch_update(const BatchRun& r, int j, const int* ngroups) {
  if (r.count <= 0) return hipSuccess;
  return batch_fp32(r) ? batch_update_t<float>(r, j, ngroups)
                       : batch_update_t<double>(r, j, ngroups);
}

hipError_t batch_lsq(const BatchRun& r, int m) {
  if (r.count <= 0) return hipSuccess;
  const int panel = lsq_panel(m);
  const size_t lds = ((size_t)m + 1 + (size_t)panel * m) * sizeof(double);
  int nb[kMaxBatch];
  for (int k = 0; k < r.count; ++k) nb[k] = 1;
  BatchMap mp;
  build_map(mp, r, nb, nullptr);
  const Inst* t = r.d_tab;
  int pa = panel;
  void* args[] = {&t, &mp, &pa};
  return launch_map(reinterpret_cast<const void*>(lsq_batch_kernel), mp, 256, lds, args, r.stream);
}

hipError_t batch_xupdate(const BatchRun& r) {
  if (r.count <= 0) return hipSuccess;
  const long long per = (long long)kUpdateThreads * kUpdateRows;
  int nb[kMaxBatch];
  for (int k = 0; k < r.count; ++k) {
    long long g = (r.h_tab[r.act[k]].n + per - 1) / per;   // as launch_xupdate
    nb[k] = (int)(g > kMaxBlocks ? kMaxBlocks : g);
  }
  BatchMap m;
  build_map(m, r, nb, nullptr);
  const Inst* t = r.d_tab;
  void* args[] = {&t, &m};
  const void* kern = batch_fp32(r) ? reinterpret_cast<const void*>(xupdate_batch_kernel<float>)
                                   : reinterpret_cast<const void*>(xupdate_batch_kernel<double>);
  return launch_map(kern, m, kUpdateThreads, 0, args, r.stream);
}

hipError_t batch_ctl_gather(const BatchRun& r, Ctl* out) {
  if (r.count <= 0) return hipSuccess;
  int nb[kMaxBatch];
  for (int k = 0; k < r.count; ++k) nb[k] = 1;
  BatchMap m;
  build_map(m, r, nb, nullptr);
  const Inst* t = r.d_tab;
  Ctl* o = out;
  void* args[] = {&t, &m, &o};
  return launch_map(reinterpret_cast<const void*>(ctl_gather_kernel), m, 64, 0, args, r.stream);
}

}  // namespace igs
