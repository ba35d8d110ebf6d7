// Host side of the C ABI (include/igs.h): contexts, workspace, the restarted
// GMRES(m) driver and per-kernel event timing.  Every arithmetic step of the
// solve runs in the kernels of kernels.hip; this file only validates input,
// allocates, queues launches and reads one small control block per cycle.
#include "../../include/igs.h"
#include "igs_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

using igs::Ctl;
using igs::Op;
using igs::Work;

namespace {

// Message of the last failing call that has no context (igs_create*, the
// serving and no-allocation entry points): a fixed buffer, so that setting it
// allocates nothing.
thread_local char g_create_error[512];

struct EventPair {
  hipEvent_t a, b;
  int kernel;
  int j;        // iteration (-1: per cycle)
  int cycle;
  int ran;      // -1: unknown until the cycle ends; 0/1 afterwards
  double bytes;
};

struct KStat {
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

// What a recorded restart cycle depends on: buffers and settings baked into
// its launches.  Zero-initialised, compared byte for byte.
struct CycleKey {
  const double* b;
  const double* x;
  const double* V;
  const float* V32;
  long long n, nnz;
  long long maxit;
  double tol, tau, cycle_rtol;
  int m, gs, final_v, fp32;
  int lpr, dense;
  int rpg, tune_gen;
  int dense_mfma, pad2;
  int fuse, pre;
};

}  // namespace

struct igs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  long long n = 0, nnz = 0;
  Op op{};
  int* d_row_ptr = nullptr;
  int* d_col = nullptr;
  double* d_vals = nullptr;
  double* d_A = nullptr;
  float* d_vals32 = nullptr;   // CSR values rounded to FP32 (first mixed-precision solve)
  int* d_ell_col = nullptr;    // the operator in column-major ELL form (short rows)
  short* d_ell_dcol = nullptr; // its column indices as 16-bit offsets from the row
  double* d_ell_val = nullptr;
  float* d_ell_val32 = nullptr;
  long long n_cap = 0, nnz_cap = 0;  // serving slot: device capacity for rebinding operators
  double es_bytes = 8.0;       // bytes of a basis element in the current solve

  // workspace for restart length m_alloc
  int m32_alloc = 0;           // columns + 1 of the FP32 basis (mixed precision)
  int m_alloc = 0;
  Work w{};
  Ctl* h_ctl = nullptr;  // pinned host copy of the control block

  // raw step-kernel scratch
  int raw_cols = 0;
  double* raw_part = nullptr;
  double* raw_gpart = nullptr;
  unsigned* raw_tickets = nullptr;
  double* raw_out = nullptr;
  double* raw_t = nullptr;
  double* raw_r1 = nullptr;

  // first-cycle snapshot
  std::vector<double> H_first;
  int J_first = -1;
  int ldh_first = 0;
  double* d_V_first = nullptr;
  size_t V_first_cols = 0;
  int V_first_valid = 0;

  // profiling
  std::vector<hipEvent_t> event_pool;   // every event created (destroyed with the context)
  std::vector<hipEvent_t> event_free;   // events ready for reuse
  std::vector<EventPair> pending;
  KStat stats[IGS_K_COUNT];

  KStat stats_j[IGS_K_COUNT][IGS_MAX_RESTART + 1];   // the same per iteration j

  // launch shapes chosen by igs_tune (empty: the defaults)
  std::vector<unsigned char> tune;
  int tune_gen = 0;

  // a restart cycle recorded in a HIP graph (opts.cycle_graph)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t cycle_exec = nullptr;
  CycleKey cycle_key{};

  std::string err;
};

namespace {

// The dense operator apply the contexts start with (igs_dense_variant changes it).
constexpr int DENSE_MFMA_DEFAULT = 0;

int set_err(igs_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else snprintf(g_create_error, sizeof g_create_error, "%s", buf);
  return code;
}

#define HIP_OR_FAIL(ctx, call)                                                                 \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      return set_err((ctx), e_ == hipErrorOutOfMemory ? IGS_ENOMEM : IGS_EDEVICE, "%s: %s",   \
                     #call, hipGetErrorString(e_));                                            \
    }                                                                                          \
  } while (0)

void free_workspace(igs_ctx* c) {
  Work& w = c->w;
  void* ptrs[] = {w.V, w.z, w.H, w.R, w.T, w.L, w.cs, w.sn, w.g, w.y, w.coef_t, w.coef_r1, w.pre,
                  w.part, w.gpart, w.tickets, w.ctl, c->d_V_first, w.V32, w.z32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  c->h_ctl = nullptr;
  c->d_V_first = nullptr;
  c->V_first_cols = 0;
  c->w = Work{};
  c->m_alloc = 0;
  c->m32_alloc = 0;
}

void free_raw(igs_ctx* c) {
  void* ptrs[] = {c->raw_part, c->raw_gpart, c->raw_tickets, c->raw_out, c->raw_t, c->raw_r1};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  c->raw_part = c->raw_gpart = c->raw_out = c->raw_t = c->raw_r1 = nullptr;
  c->raw_tickets = nullptr;
  c->raw_cols = 0;
}

// Largest singular value of the first cycle's (J+1) x J Hessenberg matrix
// (column-major, leading dimension ldh): Lanczos with full
// reorthogonalisation on H^T H (at most 100 steps, exact when J <= 100),
// then the largest eigenvalue of the Lanczos tridiagonal by bisection on its
// Sturm sequence.  With an orthonormal basis, A V_J = V_{J+1} H, so the
// result is ||A V_J||_2, a lower bound of ||A||_2 from the Krylov space the
// solve built.  A diagnostic for the caller; no step of the solve uses it.
double hessenberg_norm2(const std::vector<double>& H, int ldh, int J) {
  if (J <= 0) return NAN;
  const int kmax = std::min(J, 100);
  std::vector<double> Q((size_t)kmax * J), w((size_t)J), hv((size_t)J + 1);
  std::vector<double> al(kmax), be(kmax);
  auto apply = [&](const double* v, double* out) {   // out = H^T (H v)
    for (int i = 0; i <= J; ++i) hv[i] = 0.0;
    for (int k = 0; k < J; ++k)
      for (int i = 0; i <= k + 1 && i <= J; ++i) hv[i] += H[(size_t)k * ldh + i] * v[k];
    for (int k = 0; k < J; ++k) {
      double acc = 0.0;
      for (int i = 0; i <= k + 1 && i <= J; ++i) acc += H[(size_t)k * ldh + i] * hv[i];
      out[k] = acc;
    }
  };
  for (int i = 0; i < J; ++i) Q[i] = 1.0 / sqrt((double)J);
  int k = 0;
  for (; k < kmax; ++k) {
    const double* q = &Q[(size_t)k * J];
    apply(q, w.data());
    double a = 0.0;
    for (int i = 0; i < J; ++i) a += q[i] * w[i];
    al[k] = a;
    // full reorthogonalisation against every Lanczos vector, twice
    for (int pass = 0; pass < 2; ++pass)
      for (int l = 0; l <= k; ++l) {
        const double* ql = &Q[(size_t)l * J];
        double d = 0.0;
        for (int i = 0; i < J; ++i) d += ql[i] * w[i];
        for (int i = 0; i < J; ++i) w[i] -= d * ql[i];
      }
    double b = 0.0;
    for (int i = 0; i < J; ++i) b += w[i] * w[i];
    b = sqrt(b);
    be[k] = b;
    if (k + 1 == kmax || !(b > 1e-14 * fabs(a))) { ++k; break; }
    double* qn = &Q[(size_t)(k + 1) * J];
    for (int i = 0; i < J; ++i) qn[i] = w[i] / b;
  }
  // largest eigenvalue of the k x k tridiagonal (al, be): bisection with
  // Sturm counts on the Gershgorin interval
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i + 1 < k ? fabs(be[i]) : 0.0);
    hi = std::max(hi, al[i] + r);
    lo = std::min(lo, al[i] - r);
  }
  auto below = [&](double x) {   // eigenvalues < x
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double off = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
      d = al[i] - x - (i > 0 ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(fabs(hi), 1e-300); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) < k) lo = mid; else hi = mid;
  }
  return sqrt(std::max(0.0, 0.5 * (lo + hi)));
}

long long pick_ldv(long long n) {
  long long ld = (n + 63) / 64 * 64;
  if (ld % 4096 == 0) ld += 64;  // no large power-of-two stride between columns
  return ld;
}

int ensure_workspace(igs_ctx* c, int m) {
  if (c->m_alloc >= m) return IGS_OK;
  free_workspace(c);
  Work& w = c->w;
  const long long n = c->n;
  w.ldv = pick_ldv(n);
  w.ldh = m + 1;
  w.ldt = m + 1;
  w.pstride = (2 * (m + 1) + 7) / 8 * 8;
  if (w.pstride < 8) w.pstride = 8;
  HIP_OR_FAIL(c, dalloc(&w.V, (size_t)w.ldv * (m + 1)));
  HIP_OR_FAIL(c, dalloc(&w.z, (size_t)w.ldv));
  HIP_OR_FAIL(c, dalloc(&w.H, (size_t)m * (m + 3) / 2));
  HIP_OR_FAIL(c, dalloc(&w.R, (size_t)w.ldh * m));
  HIP_OR_FAIL(c, dalloc(&w.T, (size_t)(m + 1) * (m + 2) / 2));
  HIP_OR_FAIL(c, dalloc(&w.L, (size_t)w.ldt * w.ldt));
  HIP_OR_FAIL(c, dalloc(&w.cs, (size_t)m));
  HIP_OR_FAIL(c, dalloc(&w.sn, (size_t)m));
  HIP_OR_FAIL(c, dalloc(&w.g, (size_t)m + 1));
  HIP_OR_FAIL(c, dalloc(&w.y, (size_t)m));
  HIP_OR_FAIL(c, dalloc(&w.coef_t, (size_t)m + 2));
  HIP_OR_FAIL(c, dalloc(&w.coef_r1, (size_t)m + 2));
  HIP_OR_FAIL(c, dalloc(&w.pre, (size_t)3 * (m + 2)));
  HIP_OR_FAIL(c, dalloc(&w.part, (size_t)igs::kMaxBlocks * w.pstride));
  HIP_OR_FAIL(c, dalloc(&w.gpart, (size_t)igs::kMaxGroups * w.pstride));
  HIP_OR_FAIL(c, dalloc(&w.tickets, (size_t)igs::kMaxGroups + 1));
  HIP_OR_FAIL(c, dalloc(&w.ctl, 1));
  HIP_OR_FAIL(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_ctl), sizeof(Ctl),
                               hipHostMallocDefault));
  // Zero-fill at allocation, outside any captured work.
  HIP_OR_FAIL(c, hipMemsetAsync(w.tickets, 0, sizeof(unsigned) * (igs::kMaxGroups + 1), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(w.ctl, 0, sizeof(Ctl), c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(w.T, 0, sizeof(double) * (m + 1) * (m + 2) / 2, c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(w.L, 0, sizeof(double) * w.ldt * w.ldt, c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(w.H, 0, sizeof(double) * m * (m + 3) / 2, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  memset(c->h_ctl, 0, sizeof(Ctl));
  c->m_alloc = m;
  return IGS_OK;
}

// FP32 basis and A u (same leading dimension as the FP64 basis) and the FP32
// copy of the CSR values, for the mixed-precision cycles.
int ensure_fp32(igs_ctx* c, int m) {
  Work& w = c->w;
  if (!c->d_vals32 && c->nnz > 0) {
    // a serving slot sizes the copy for the largest operator it will hold
    const long long nv = c->nnz_cap > c->nnz ? c->nnz_cap : c->nnz;
    float* v = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&v), sizeof(float) * nv) != hipSuccess)
      return set_err(c, IGS_ENOMEM, "cannot allocate %lld FP32 operator values", nv);
    c->d_vals32 = v;
    HIP_OR_FAIL(c, igs::launch_round_to_float(c->d_vals, c->d_vals32, c->nnz, c->stream));
    c->op.vals32 = c->d_vals32;
  }
  if (c->op.ell_k > 0 && !c->d_ell_val32) {
    const long long ne = (long long)c->op.ell_k * c->n;
    float* v = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&v), sizeof(float) * ne) != hipSuccess)
      return set_err(c, IGS_ENOMEM, "cannot allocate %lld FP32 ELL values", ne);
    c->d_ell_val32 = v;
    HIP_OR_FAIL(c, igs::launch_round_to_float(c->d_ell_val, c->d_ell_val32, ne, c->stream));
    c->op.ell_val32 = c->d_ell_val32;
  }
  if (c->m32_alloc >= m + 1 && w.V32) return IGS_OK;
  if (w.V32) (void)hipFree(w.V32);
  if (w.z32) (void)hipFree(w.z32);
  w.V32 = nullptr;
  w.z32 = nullptr;
  c->m32_alloc = 0;
  if (hipMalloc(reinterpret_cast<void**>(&w.V32), sizeof(float) * w.ldv * (m + 1)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w.z32), sizeof(float) * w.ldv) != hipSuccess)
    return set_err(c, IGS_ENOMEM, "cannot allocate the FP32 basis (%lld x %d)", w.ldv, m + 1);
  c->m32_alloc = m + 1;
  return IGS_OK;
}

int ensure_raw(igs_ctx* c, int cols) {
  if (c->raw_cols >= cols) return IGS_OK;
  free_raw(c);
  const int pstride = (2 * cols + 7) / 8 * 8;
  HIP_OR_FAIL(c, dalloc(&c->raw_part, (size_t)igs::kMaxBlocks * pstride));
  HIP_OR_FAIL(c, dalloc(&c->raw_gpart, (size_t)igs::kMaxGroups * pstride));
  HIP_OR_FAIL(c, dalloc(&c->raw_tickets, (size_t)igs::kMaxGroups + 1));
  HIP_OR_FAIL(c, dalloc(&c->raw_out, (size_t)2 * cols));
  HIP_OR_FAIL(c, dalloc(&c->raw_t, (size_t)cols + 1));
  HIP_OR_FAIL(c, dalloc(&c->raw_r1, (size_t)cols + 1));
  HIP_OR_FAIL(c, hipMemsetAsync(c->raw_tickets, 0, sizeof(unsigned) * (igs::kMaxGroups + 1),
                                c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->raw_cols = cols;
  return IGS_OK;
}

// ---- profiling ------------------------------------------------------------

hipEvent_t next_event(igs_ctx* c) {
  if (!c->event_free.empty()) {
    hipEvent_t e = c->event_free.back();
    c->event_free.pop_back();
    return e;
  }
  hipEvent_t e;
  // timing events without the system-scope fence: the times are read by the
  // host after a stream synchronisation, never through host-visible memory
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  c->event_pool.push_back(e);
  return e;
}

struct Timed {
  igs_ctx* c;
  bool on;
  EventPair p{};
  Timed(igs_ctx* c_, int mask, int kernel, int j, int cycle, double bytes)
      : c(c_), on((mask >> kernel) & 1) {
    if (!on) return;
    p.a = next_event(c);
    p.b = next_event(c);
    p.kernel = kernel;
    p.j = j;
    p.cycle = cycle;
    p.ran = -1;
    p.bytes = bytes;
    if (p.a) (void)hipEventRecord(p.a, c->stream);
  }
  ~Timed() {
    if (!on || !p.a || !p.b) return;
    (void)hipEventRecord(p.b, c->stream);
    c->pending.push_back(p);
  }
};

// Did launch (kernel, j) of a cycle that ended at iteration j_end do work?
bool launch_ran(int kernel, int j, int j_end, int m) {
  switch (kernel) {
    case IGS_K_SPMV: return j <= j_end && j < m;
    case IGS_K_OPREDUCE: return j <= j_end && j < m;
    case IGS_K_REDUCE: return j <= j_end;
    case IGS_K_UPDATE: return j <= j_end;
    default: return true;
  }
}

// At the end of a cycle: record which of its launches did work.  The event
// times themselves are read later (harvest), outside any timed loop.
void mark_cycle(igs_ctx* c, int j_end, int m, int J, double dn) {
  for (EventPair& p : c->pending) {
    if (p.ran >= 0) continue;  // launches of earlier cycles are already marked
    bool ran = launch_ran(p.kernel, p.j, j_end, m);
    if (p.kernel == IGS_K_XUPDATE) {
      ran = J > 0;
      p.bytes = c->es_bytes * dn * J + 16.0 * dn;
    }
    p.ran = ran ? 1 : 0;
  }
}

// Read the times of every launch of finished cycles (ran >= 0) and recycle
// their events.  Called while the GPU works on the next cycle, so the reads
// never stall it; with wait = true (igs_profile_get) everything is drained.
void harvest(igs_ctx* c, bool wait) {
  if (wait) (void)hipStreamSynchronize(c->stream);
  size_t keep = 0;
  for (size_t k = 0; k < c->pending.size(); ++k) {
    EventPair& p = c->pending[k];
    if (p.ran < 0 && !wait) {
      c->pending[keep++] = p;
      continue;
    }
    if (p.ran == 1) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        KStat& s = c->stats[p.kernel];
        s.launches += 1;
        s.ms += ms;
        s.bytes += p.bytes;
        if (p.j >= 0 && p.j <= IGS_MAX_RESTART) {
          KStat& sj = c->stats_j[p.kernel][p.j];
          sj.launches += 1;
          sj.ms += ms;
          sj.bytes += p.bytes;
        }
      }
    }
    c->event_free.push_back(p.a);
    c->event_free.push_back(p.b);
  }
  c->pending.resize(keep);
}

int validate_csr(igs_ctx* c, long long n, long long nnz, const int32_t* rp, const int32_t* ci,
                 const double* va) {
  if (rp[0] != 0) return set_err(c, IGS_EINVAL, "row_ptr[0] = %d, expected 0", rp[0]);
  for (long long i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return set_err(c, IGS_EINVAL, "row_ptr decreases at row %lld", i);
  if ((long long)rp[n] != nnz)
    return set_err(c, IGS_EINVAL, "row_ptr[n] = %d, expected nnz = %lld", rp[n], nnz);
  for (long long k = 0; k < nnz; ++k) {
    if (ci[k] < 0 || (long long)ci[k] >= n)
      return set_err(c, IGS_EINVAL, "col_idx[%lld] = %d out of range", k, ci[k]);
    if (!isfinite(va[k])) return set_err(c, IGS_EINVAL, "vals[%lld] is not finite", k);
  }
  return IGS_OK;
}

int common_create(igs_ctx** out, void* hip_stream, igs_ctx** made) {
  if (!out) return set_err(nullptr, IGS_EINVAL, "out is NULL");
  *out = nullptr;
  igs_ctx* c = new (std::nothrow) igs_ctx();
  if (!c) return set_err(nullptr, IGS_ENOMEM, "host allocation failed");
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return set_err(nullptr, IGS_EDEVICE, "no HIP device");
  }
  *made = c;
  return IGS_OK;
}

int fail_create(igs_ctx* c, int code) {
  snprintf(g_create_error, sizeof g_create_error, "%s", c->err.c_str());
  igs_destroy(c);
  return code;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" int igs_create(igs_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                          const int32_t* col_idx, const double* vals, int ptrs_on_device,
                          void* hip_stream) {
  if (n < 1 || nnz < 0 || !row_ptr || (nnz > 0 && (!col_idx || !vals)))
    return set_err(nullptr, IGS_EINVAL, "invalid size or NULL array");
  if (n >= (1LL << 31) || nnz >= (1LL << 31))
    return set_err(nullptr, IGS_EINVAL, "n and nnz must fit int32 indexing");
  igs_ctx* c = nullptr;
  int rc = common_create(out, hip_stream, &c);
  if (rc != IGS_OK) return rc;
  c->n = n;
  c->nnz = nnz;
  // host copies for validation (and staging of device input)
  std::vector<int32_t> hrp, hci;
  std::vector<double> hva;
  const int32_t* rp = row_ptr;
  const int32_t* ci = col_idx;
  const double* va = vals;
  if (ptrs_on_device) {
    hrp.resize(n + 1);
    hci.resize(nnz);
    hva.resize(nnz);
    if (hipMemcpy(hrp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        (nnz > 0 && (hipMemcpy(hci.data(), col_idx, sizeof(int32_t) * nnz,
                               hipMemcpyDeviceToHost) != hipSuccess ||
                     hipMemcpy(hva.data(), vals, sizeof(double) * nnz, hipMemcpyDeviceToHost) !=
                         hipSuccess))) {
      set_err(c, IGS_EINVAL, "could not read the CSR arrays from device memory");
      return fail_create(c, IGS_EINVAL);
    }
    rp = hrp.data();
    ci = hci.data();
    va = hva.data();
  }
  rc = validate_csr(c, n, nnz, rp, ci, va);
  if (rc != IGS_OK) return fail_create(c, rc);
  if (dalloc(&c->d_row_ptr, n + 1) != hipSuccess || dalloc(&c->d_col, nnz) != hipSuccess ||
      dalloc(&c->d_vals, nnz) != hipSuccess) {
    set_err(c, IGS_ENOMEM, "device allocation of the operator failed");
    return fail_create(c, IGS_ENOMEM);
  }
  const hipMemcpyKind kind = ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (hipMemcpy(c->d_row_ptr, row_ptr, sizeof(int32_t) * (n + 1), kind) != hipSuccess ||
      (nnz > 0 && (hipMemcpy(c->d_col, col_idx, sizeof(int32_t) * nnz, kind) != hipSuccess ||
                   hipMemcpy(c->d_vals, vals, sizeof(double) * nnz, kind) != hipSuccess))) {
    set_err(c, IGS_EDEVICE, "copy of the operator to the device failed");
    return fail_create(c, IGS_EDEVICE);
  }
  // lanes per row: the power of two at or above the mean row length
  const double avg = (double)nnz / (double)n;
  int lpr = 1;
  while (lpr < 64 && (double)lpr < avg) lpr *= 2;
  c->op.dense = 0;
  c->op.n = n;
  c->op.row_ptr = c->d_row_ptr;
  c->op.col_idx = c->d_col;
  c->op.vals = c->d_vals;
  c->op.lpr = lpr;
  // Rows of at most 8 entries with 8 lanes per row (stencils): also keep the
  // column-major ELL form, whose product is bit-identical and one memory
  // latency shorter.
  if (lpr == 8) {
    long long kmax = 0;
    for (long long i = 0; i < n; ++i) kmax = std::max<long long>(kmax, rp[i + 1] - rp[i]);
    if (kmax >= 1 && kmax <= 8) {
      std::vector<int32_t> ec((size_t)kmax * n, 0);
      std::vector<double> ev((size_t)kmax * n, 0.0);
      for (long long i = 0; i < n; ++i)
        for (long long k = rp[i]; k < rp[i + 1]; ++k) {
          ec[(size_t)(k - rp[i]) * n + i] = ci[k];
          ev[(size_t)(k - rp[i]) * n + i] = va[k];
        }
      if (dalloc(&c->d_ell_col, (size_t)kmax * n) != hipSuccess ||
          dalloc(&c->d_ell_val, (size_t)kmax * n) != hipSuccess ||
          hipMemcpy(c->d_ell_col, ec.data(), sizeof(int32_t) * kmax * n, hipMemcpyHostToDevice) !=
              hipSuccess ||
          hipMemcpy(c->d_ell_val, ev.data(), sizeof(double) * kmax * n, hipMemcpyHostToDevice) !=
              hipSuccess) {
        set_err(c, IGS_ENOMEM, "device allocation of the ELL form failed");
        return fail_create(c, IGS_ENOMEM);
      }
      c->op.ell_k = (int)kmax;
      c->op.ell_col = c->d_ell_col;
      c->op.ell_val = c->d_ell_val;
      // the same indices as offsets from the row, when all fit 16 bits
      bool narrow = true;
      for (long long i = 0; i < n && narrow; ++i)
        for (long long k = rp[i]; k < rp[i + 1]; ++k)
          if (ci[k] - i > 32767 || ci[k] - i < -32767) {
            narrow = false;
            break;
          }
      if (narrow) {
        std::vector<int16_t> ed((size_t)kmax * n, 0);
        for (long long i = 0; i < n; ++i)
          for (long long k = rp[i]; k < rp[i + 1]; ++k)
            ed[(size_t)(k - rp[i]) * n + i] = (int16_t)(ci[k] - i);
        if (dalloc(&c->d_ell_dcol, (size_t)kmax * n) != hipSuccess ||
            hipMemcpy(c->d_ell_dcol, ed.data(), sizeof(int16_t) * kmax * n,
                      hipMemcpyHostToDevice) != hipSuccess) {
          set_err(c, IGS_ENOMEM, "device allocation of the ELL offsets failed");
          return fail_create(c, IGS_ENOMEM);
        }
        c->op.ell_dcol = c->d_ell_dcol;
      }
    }
  }
  *out = c;
  return IGS_OK;
}

extern "C" int igs_create_dense(igs_ctx** out, int64_t n, const double* A, int64_t lda,
                                int ptr_on_device, void* hip_stream) {
  if (n < 1 || !A || lda < n) return set_err(nullptr, IGS_EINVAL, "invalid size or NULL array");
  if (n >= (1LL << 31)) return set_err(nullptr, IGS_EINVAL, "n too large");
  igs_ctx* c = nullptr;
  int rc = common_create(out, hip_stream, &c);
  if (rc != IGS_OK) return rc;
  c->n = n;
  c->nnz = n * n;
  const long long ldd = (n + 63) / 64 * 64;
  std::vector<double> host;
  const double* src = A;
  if (ptr_on_device) {
    host.resize((size_t)n * lda);
    if (hipMemcpy(host.data(), A, sizeof(double) * n * lda, hipMemcpyDeviceToHost) !=
        hipSuccess) {
      set_err(c, IGS_EINVAL, "could not read A from device memory");
      return fail_create(c, IGS_EINVAL);
    }
    src = host.data();
  }
  for (long long i = 0; i < n; ++i)
    for (long long k = 0; k < n; ++k)
      if (!isfinite(src[i * lda + k])) {
        set_err(c, IGS_EINVAL, "A[%lld, %lld] is not finite", i, k);
        return fail_create(c, IGS_EINVAL);
      }
  if (dalloc(&c->d_A, (size_t)n * ldd) != hipSuccess) {
    set_err(c, IGS_ENOMEM, "device allocation of A failed");
    return fail_create(c, IGS_ENOMEM);
  }
  // zeros in the padding columns: the matrix-core kernel reads whole steps
  // of 32 columns
  if (hipMemset(c->d_A, 0, sizeof(double) * n * ldd) != hipSuccess) {
    set_err(c, IGS_EDEVICE, "clearing A on the device failed");
    return fail_create(c, IGS_EDEVICE);
  }
  if (hipMemcpy2D(c->d_A, ldd * sizeof(double), src, lda * sizeof(double), n * sizeof(double), n,
                  hipMemcpyHostToDevice) != hipSuccess) {
    set_err(c, IGS_EDEVICE, "copy of A to the device failed");
    return fail_create(c, IGS_EDEVICE);
  }
  c->op.dense = 1;
  c->op.n = n;
  c->op.A = c->d_A;
  c->op.lda = ldd;
  c->op.dense_mfma = DENSE_MFMA_DEFAULT;
  *out = c;
  return IGS_OK;
}

extern "C" int igs_destroy(igs_ctx* c) {
  if (!c) return IGS_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_workspace(c);
  free_raw(c);
  void* ptrs[] = {c->d_row_ptr, c->d_col, c->d_vals, c->d_A, c->d_vals32, c->d_ell_col,
                  c->d_ell_val, c->d_ell_val32, c->d_ell_dcol};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->cycle_exec) (void)hipGraphExecDestroy(c->cycle_exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
  return IGS_OK;
}

extern "C" const char* igs_last_error(const igs_ctx* c) {
  return c ? c->err.c_str() : g_create_error;
}

extern "C" int igs_solve(igs_ctx* c, const double* b, double* x, int restart, double tol,
                         int gs_iters, igs_info* info) {
  return igs_solve_opts(c, b, x, restart, tol, gs_iters, nullptr, info);
}

namespace {

// A restart cycle counts as stagnant (igs_info.stagnant_cycles) when the true
// residual ||b - A x|| at the start of the next cycle is above
// (1 - kStagnationDrop) times its value at the cycle's own start.  A cycle
// whose start or end residual is not finite is not counted.
constexpr double kStagnationDrop = 1e-3;

bool cycle_stagnated(double rho_start, double rho_next) {
  return isfinite(rho_start) && isfinite(rho_next) && rho_start > 0.0 &&
         rho_next > (1.0 - kStagnationDrop) * rho_start;
}

// Record the launches `enqueue` makes into the context's cycle graph.
template <typename F>
int record_cycle(igs_ctx* c, F&& enqueue) {
  if (!c->cap_stream)
    HIP_OR_FAIL(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  if (c->cycle_exec) {
    (void)hipGraphExecDestroy(c->cycle_exec);
    c->cycle_exec = nullptr;
  }
  c->cycle_key = CycleKey{};
  HIP_OR_FAIL(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue(c->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (rc != IGS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIP_OR_FAIL(c, e);
  const hipError_t ie = hipGraphInstantiate(&c->cycle_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) c->cycle_exec = nullptr;
  HIP_OR_FAIL(c, ie);
  return IGS_OK;
}

}  // namespace

extern "C" int igs_solve_opts(igs_ctx* c, const double* b, double* x, int restart, double tol,
                              int gs_iters, const igs_opts* opts, igs_info* info) {
  if (!c) return IGS_EINVAL;
  c->err.clear();
  if (!b || !x) return set_err(c, IGS_EINVAL, "b and x must be device pointers");
  if ((reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(x)) % 16 != 0)
    return set_err(c, IGS_EINVAL, "b and x must be 16-byte aligned");
  if (restart < 1) return set_err(c, IGS_EINVAL, "restart must be >= 1");
  if (!(tol >= 0.0) || !isfinite(tol)) return set_err(c, IGS_EINVAL, "tol must be finite, >= 0");
  if (gs_iters != 1 && gs_iters != 2) return set_err(c, IGS_EINVAL, "gs_iters must be 1 or 2");
  igs_opts o{};
  if (opts) o = *opts;
  const auto t0 = std::chrono::steady_clock::now();
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const long long n = c->n;
  int m = restart;
  if (m > n) m = (int)n;
  if (m > IGS_MAX_RESTART) m = IGS_MAX_RESTART;
  int rc = ensure_workspace(c, m);
  if (rc != IGS_OK) return rc;
  const long long maxit = o.maxit > 0 ? o.maxit : 20 * n;
  const double tau = o.lagnorm_tau > 0.0 ? o.lagnorm_tau : 1e-4;
  const bool mgs = o.mgs != 0;
  const bool prof = o.profile != 0 && !mgs;
  const int pmask = prof ? (o.profile_kernels ? o.profile_kernels : (1 << IGS_K_COUNT) - 1) : 0;
  const int final_v = o.final_basis_vector ? 1 : 0;
  const bool fp32 = o.inner_fp32 != 0;
  const bool fuse = o.separate_apply == 0;
  // two-reduce with two sweeps: the one-sweep step plus a second reduction
  // and correction per iteration
  const bool two_reduce = o.two_reduce != 0 && gs_iters == 2;
  const int gs_step = two_reduce ? 1 : gs_iters;
  const double cycle_rtol = fp32 ? (o.inner_rtol > 0.0 ? o.inner_rtol : 1e-5) : 0.0;
  if (mgs && (fp32 || o.two_reduce))
    return set_err(c, IGS_ENOTIMPL, "the MGS comparator is FP64 and one-pass only");
  if (fp32) {
    if (c->op.dense) return set_err(c, IGS_ENOTIMPL, "FP32 cycles need a CSR operator");
    if (o.keep_first_basis)
      return set_err(c, IGS_ENOTIMPL, "keep_first_basis is FP64 only (the basis is FP32)");
    rc = ensure_fp32(c, m);
    if (rc != IGS_OK) return rc;
  }
  Work& w = c->w;
  w.fp32 = fp32 ? 1 : 0;
  w.tune = c->tune.empty() ? nullptr : c->tune.data();
  // the small products of large iterations in a kernel of their own
  w.pre_on = o.products_in_update ? 0 : 1;
  w.col_split = c->op.dense ? 1 : 0;
  hipStream_t s = c->stream;
  c->J_first = -1;
  c->V_first_valid = 0;

  // ||b|| and the finiteness of b and x0
  HIP_OR_FAIL(c, igs::launch_bnorm(b, x, n, w, s));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->h_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(c, hipStreamSynchronize(s));
  if (c->h_ctl->nonfinite_in > 0)
    return set_err(c, IGS_EINVAL, "b or x0 holds %d non-finite entries", c->h_ctl->nonfinite_in);
  const double bnorm = c->h_ctl->bnorm;

  // algorithmic bytes of each launch (minimum HBM traffic of its shape);
  // es: bytes of a basis element (8, or 4 in FP32 cycles)
  const double dn = (double)n;
  const double es = fp32 ? 4.0 : 8.0;
  const double op64_bytes = c->op.dense ? 8.0 * dn * dn + 16.0 * dn
                                        : 12.0 * (double)c->nnz + 4.0 * (dn + 1) + 16.0 * dn;
  const double op_bytes = fp32 ? 8.0 * (double)c->nnz + 4.0 * (dn + 1) + 2.0 * es * dn
                               : op64_bytes;
  c->es_bytes = es;

  long long its = 0;
  int cycles = 0;
  int status = igs::kRunning;
  int ret = IGS_ENOCONV;
  double relres = NAN, arn = NAN;
  double rho_prev = NAN;   // ||b - A x|| at the start of the previous cycle
  int stagnant = 0;
  bool converged = false;
  bool final_check = false;
  int cycles_timed = 0;   // the cycle index the profiling events carry
  // The launches of one restart cycle on stream `st`: the residual, the
  // iterations 0..jmax, then the least squares and x update.  A check cycle
  // (after the iteration budget) runs iteration 0 only: the residual norm
  // decides between convergence and giving up.  its_before < 0: the cycle
  // takes the count the host wrote into the control block (graph replay).
  auto enqueue_cycle = [&](hipStream_t st, long long its_before, long long maxit_cycle,
                           bool check) -> int {
    if (mgs) {
      // modified Gram-Schmidt: v_0 = r0 / ||r0||, then per column c the
      // operator apply into V[:, c+1] and c + 2 reductions
      HIP_OR_FAIL(c, igs::launch_residual(c->op, b, x, w, its_before, maxit_cycle, m, 1, 0, tol,
                                          tau, 0.0, st));
      HIP_OR_FAIL(c, igs::launch_mgs_start(w, n, st));
      if (check) return IGS_OK;
      for (int col = 0; col < m; ++col) {
        HIP_OR_FAIL(c, igs::launch_spmv(c->op, w.V + (size_t)col * w.ldv,
                                        w.V + (size_t)(col + 1) * w.ldv, w.ctl, col, st));
        HIP_OR_FAIL(c, igs::launch_mgs_column(w, n, col, st));
      }
      HIP_OR_FAIL(c, igs::launch_lsq(w, m, st));
      HIP_OR_FAIL(c, igs::launch_xupdate(w, n, x, st));
      return IGS_OK;
    }
    {
      Timed tm(c, pmask, IGS_K_RESIDUAL, -1, cycles_timed, op64_bytes + es * dn);
      HIP_OR_FAIL(c, igs::launch_residual(c->op, b, x, w, its_before, maxit_cycle, m, gs_step,
                                          final_v, tol, tau, cycle_rtol, st));
    }
    const int jmax = check ? 0 : m;
    for (int j = 0; j <= jmax; ++j) {
      // the operator apply inside the reduction's blocks where it fits,
      // else as a kernel of its own before it (the same results either way)
      const bool fused = fuse && j < m && igs::opreduce_fits(c->op, w, n, j);
      if (j < m && !fused) {
        Timed tm(c, pmask, IGS_K_SPMV, j, cycles_timed, op_bytes);
        if (fp32)
          HIP_OR_FAIL(c, igs::launch_spmv32(c->op, w.V32 + (size_t)j * w.ldv, w.z32, w.ctl, j, st));
        else
          HIP_OR_FAIL(c, igs::launch_spmv(c->op, w.V + (size_t)j * w.ldv, w.z, w.ctl, j, st));
      }
      int nb = 0;
      if (fused) {
        // the operator's arrays and z written once; u read once, as column j
        Timed tm(c, pmask, IGS_K_OPREDUCE, j, cycles_timed,
                 op_bytes - es * dn + es * dn * (j + 1));
        HIP_OR_FAIL(c, igs::launch_opreduce(c->op, w, n, j, st, &nb));
      } else {
        Timed tm(c, pmask, IGS_K_REDUCE, j, cycles_timed,
                 es * dn * (j + 1) + (j < m ? es * dn : 0.0));
        HIP_OR_FAIL(c, igs::launch_reduce(w, n, j, j < m, st, &nb));
      }
      // The update kernel runs the small solve of iteration j in every block.
      // The tail update (j = m) finishes the last column (and the lagged-norm
      // fallback there) and writes v_m on request; it never writes column
      // m + 1.
      if (igs::coef_kernel_needed(w, j))
        HIP_OR_FAIL(c, igs::launch_coef(w, j, igs::reduce_groups(nb), st));
      {
        Timed tm(c, pmask, IGS_K_UPDATE, j, cycles_timed, es * dn * (j + 1) + 3.0 * es * dn);
        HIP_OR_FAIL(c, igs::launch_update(w, n, j, gs_step, igs::reduce_groups(nb), st));
      }
      if (two_reduce && j < m && !check) {
        // second sweep on u_{j+1}: r2 = [V_{0:j+1}, u]^T u, then the correction
        int nb2 = 0;
        HIP_OR_FAIL(c, igs::launch_reduce(w, n, j + 1, false, st, &nb2));
        HIP_OR_FAIL(c, igs::launch_correct(w, n, j + 1, igs::reduce_groups(nb2), st));
      }
    }
    if (!check) {
      HIP_OR_FAIL(c, igs::launch_lsq(w, m, st));
      Timed tm(c, pmask, IGS_K_XUPDATE, -1, cycles_timed, 0.0);
      HIP_OR_FAIL(c, igs::launch_xupdate(w, n, x, st));
    }
    return IGS_OK;
  };
  // Graph replay of the full cycles: recorded once (on a capture stream of
  // the context, nothing runs while recording) for these settings and
  // buffers, then launched on the solver's stream after the host writes the
  // cycle's iteration count into the control block.
  const bool graph_ok = o.cycle_graph != 0 && !prof && !two_reduce && !mgs;
  CycleKey key{};
  key.b = b;
  key.x = x;
  key.V = w.V;
  key.V32 = w.V32;
  key.n = n;
  key.nnz = c->nnz;
  key.lpr = c->op.lpr;
  key.dense = c->op.dense;
  key.rpg = c->op.rpg;
  key.dense_mfma = c->op.dense_mfma;
  key.tune_gen = c->tune_gen;
  key.m = m;
  key.gs = gs_step;
  key.final_v = final_v;
  key.fp32 = fp32 ? 1 : 0;
  key.tol = tol;
  key.tau = tau;
  key.cycle_rtol = cycle_rtol;
  key.maxit = maxit;
  key.fuse = fuse ? 1 : 0;
  key.pre = w.pre_on;
  // After a cycle whose Arnoldi residual met the tolerance, the next cycle
  // is a check cycle too (its residual and iteration 0 only): the true
  // residual nearly always confirms convergence there, and a full cycle's
  // remaining launches would only return at once.  If it does not, a full
  // cycle follows.
  bool probe = false;
  bool skip_stagnation = false;   // a full cycle after a failed probe starts where the probe did
  while (true) {
    const long long its_before = its;
    const bool check = final_check || probe;
    const long long maxit_cycle = check ? its : maxit;  // a check cycle runs iteration 0 only
    cycles_timed = cycles;
    if (graph_ok && !check) {
      if (!c->cycle_exec || memcmp(&c->cycle_key, &key, sizeof(CycleKey)) != 0) {
        rc = record_cycle(c, [&](hipStream_t st) { return enqueue_cycle(st, -1, maxit, false); });
        if (rc != IGS_OK) return rc;
        c->cycle_key = key;
      }
      c->h_ctl->its_before = its_before;
      HIP_OR_FAIL(c, hipMemcpyAsync(&w.ctl->its_before, &c->h_ctl->its_before, sizeof(long long),
                                    hipMemcpyHostToDevice, s));
      HIP_OR_FAIL(c, hipGraphLaunch(c->cycle_exec, s));
    } else {
      rc = enqueue_cycle(s, its_before, maxit_cycle, check);
      if (rc != IGS_OK) return rc;
    }
    HIP_OR_FAIL(c, hipMemcpyAsync(c->h_ctl, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    if (prof) harvest(c, false);  // earlier cycles, while this one runs
    HIP_OR_FAIL(c, hipStreamSynchronize(s));
    const Ctl h = *c->h_ctl;
    status = h.status;
    const int J = h.J;
    if (prof) {
      // the iteration at which the cycle ended (every cycle ends by its tail)
      const int j_end = (h.end_iter == igs::kNotEnded) ? m : h.end_iter;
      mark_cycle(c, j_end, m, check ? 0 : J, dn);
    }
    if (cycles == 0 && !check) {
      c->J_first = J;
      c->ldh_first = w.ldh;
      if (J > 0) {
        // H is packed by columns on the device: column k holds rows 0..k+1
        const size_t packed = (size_t)J * (J + 3) / 2;
        std::vector<double> hp(packed);
        HIP_OR_FAIL(c, hipMemcpy(hp.data(), w.H, sizeof(double) * packed, hipMemcpyDeviceToHost));
        c->H_first.assign((size_t)w.ldh * J, 0.0);
        for (int k = 0; k < J; ++k)
          for (int i = 0; i <= k + 1; ++i)
            c->H_first[(size_t)k * w.ldh + i] = hp[(size_t)k * (k + 3) / 2 + i];
      }
      if (o.keep_first_basis) {
        const size_t cols = (size_t)J + 1;
        if (c->V_first_cols < cols) {
          if (c->d_V_first) (void)hipFree(c->d_V_first);
          c->d_V_first = nullptr;
          c->V_first_cols = 0;
          HIP_OR_FAIL(c, dalloc(&c->d_V_first, (size_t)w.ldv * cols));
          c->V_first_cols = cols;
        }
        HIP_OR_FAIL(c, hipMemcpyAsync(c->d_V_first, w.V, sizeof(double) * w.ldv * cols,
                                      hipMemcpyDeviceToDevice, s));
        HIP_OR_FAIL(c, hipStreamSynchronize(s));
        c->V_first_valid = 1;
      }
    }
    cycles += 1;
    relres = bnorm > 0 ? h.rho / bnorm : h.rho;
    if (!skip_stagnation && cycle_stagnated(rho_prev, h.rho)) stagnant += 1;
    skip_stagnation = false;
    rho_prev = h.rho;
    if (status == igs::kConvStart) {
      converged = true;
      ret = IGS_OK;
      break;
    }
    if (status == igs::kNonfinite) {
      ret = set_err(c, IGS_ENUMERIC, "a non-finite value appeared in cycle %d", cycles);
      its += J;
      break;
    }
    if (final_check) {
      ret = IGS_ENOCONV;
      break;
    }
    if (probe) {
      // the true residual is still above the tolerance: a full cycle from
      // the same x
      probe = false;
      skip_stagnation = true;
      continue;
    }
    its += J;
    arn = bnorm > 0 ? h.gabs / bnorm : h.gabs;
    if (J == 0) {
      ret = set_err(c, IGS_ENUMERIC, "restart cycle %d made no progress", cycles);
      break;
    }
    if (its >= maxit || (o.max_cycles > 0 && cycles >= o.max_cycles)) final_check = true;
    else if (status == igs::kConverged && h.gabs <= h.tol_abs) probe = true;
  }
  if (info) {
    info->iters = its;
    info->cycles = cycles;
    info->relres_true = relres;
    info->arnoldi_relres = arn;
    info->bnorm = bnorm;
    info->converged = converged ? 1 : 0;
    info->breakdowns = c->h_ctl->breakdowns;
    info->lagnorm_fallbacks = c->h_ctl->fallbacks;
    info->stagnant_cycles = stagnant;
    info->last_cycle_status = status;
    info->first_cycle_J = c->J_first;
    info->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (ret == IGS_ENOCONV) set_err(c, IGS_ENOCONV, "not converged after %lld iterations", its);
  return ret;
}

extern "C" int igs_debug_copy_H(igs_ctx* c, double* H_host, int ldh, int* ncols) {
  if (!c || !H_host || !ncols) return IGS_EINVAL;
  if (c->J_first < 0) return set_err(c, IGS_EINVAL, "no solve has run");
  const int J = c->J_first;
  if (ldh < J + 1) return set_err(c, IGS_EINVAL, "ldh must be >= J + 1 = %d", J + 1);
  for (int col = 0; col < J; ++col)
    for (int i = 0; i <= J; ++i)
      H_host[(size_t)col * ldh + i] = (i <= col + 1) ? c->H_first[(size_t)col * c->ldh_first + i] : 0.0;
  *ncols = J;
  return IGS_OK;
}

extern "C" int igs_dense_variant(igs_ctx* c, int variant) {
  if (!c) return IGS_EINVAL;
  if (!c->op.dense) return set_err(c, IGS_EINVAL, "not a dense operator");
  if (variant != IGS_DENSE_VALU && variant != IGS_DENSE_MFMA && variant != IGS_DENSE_LDS)
    return set_err(c, IGS_EINVAL, "variant must be IGS_DENSE_VALU, IGS_DENSE_MFMA or IGS_DENSE_LDS");
  if (variant == IGS_DENSE_LDS && c->op.lda > igs::kGemvLdsMax)
    return set_err(c, IGS_EINVAL, "IGS_DENSE_LDS holds at most %lld columns in shared memory",
                   (long long)igs::kGemvLdsMax);
  c->op.dense_mfma = variant;
  return IGS_OK;
}

extern "C" int igs_anorm_estimate(igs_ctx* c, double* out) {
  if (!c || !out) return IGS_EINVAL;
  if (c->J_first <= 0) return set_err(c, IGS_EINVAL, "no finished column in a first cycle");
  *out = hessenberg_norm2(c->H_first, c->ldh_first, c->J_first);
  return IGS_OK;
}

extern "C" int igs_debug_copy_V(igs_ctx* c, double* V_dev, int64_t ldv, int* ncols) {
  if (!c || !V_dev || !ncols) return IGS_EINVAL;
  if (!c->V_first_valid) return set_err(c, IGS_EINVAL, "solve with keep_first_basis = 1 first");
  if (ldv < c->n) return set_err(c, IGS_EINVAL, "ldv must be >= n");
  const int cols = c->J_first + 1;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, hipMemcpy2DAsync(V_dev, ldv * sizeof(double), c->d_V_first,
                                  c->w.ldv * sizeof(double), c->n * sizeof(double), cols,
                                  hipMemcpyDeviceToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  *ncols = cols;
  return IGS_OK;
}

extern "C" int igs_kernel_spmv(igs_ctx* c, const double* u, double* z) {
  if (!c || !u || !z) return IGS_EINVAL;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  HIP_OR_FAIL(c, igs::launch_spmv(c->op, u, z, nullptr, 0, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return IGS_OK;
}

extern "C" int igs_kernel_reduce(igs_ctx* c, const double* V, int64_t ldv, int j, const double* z,
                                 double* P_host, double* Q_host) {
  if (!c || !V || !P_host || j < 0 || j >= IGS_MAX_RESTART || ldv < c->n) return IGS_EINVAL;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int rc = ensure_raw(c, j + 1);
  if (rc != IGS_OK) return rc;
  const int pstride = (2 * c->raw_cols + 7) / 8 * 8;
  HIP_OR_FAIL(c, igs::launch_reduce_raw(V, ldv, c->n, j, z, c->raw_part, c->raw_gpart, pstride,
                                        c->raw_tickets, c->raw_out, c->stream));
  std::vector<double> out((size_t)2 * (j + 1));
  HIP_OR_FAIL(c, hipMemcpyAsync(out.data(), c->raw_out, sizeof(double) * out.size(),
                                hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k <= j; ++k) {
    P_host[k] = out[k];
    if (Q_host) Q_host[k] = out[(size_t)(j + 1) + k];
  }
  return IGS_OK;
}

extern "C" int igs_kernel_update(igs_ctx* c, double* V, int64_t ldv, int j, const double* z,
                                 const double* t_host, const double* r1_host, double inv_gamma) {
  if (!c || !V || !z || !r1_host || j < 0 || j >= IGS_MAX_RESTART || ldv < c->n)
    return IGS_EINVAL;
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  int rc = ensure_raw(c, j + 1);
  if (rc != IGS_OK) return rc;
  std::vector<double> tt((size_t)j + 1, 0.0);
  if (t_host)
    for (int k = 0; k < j; ++k) tt[k] = t_host[k];
  HIP_OR_FAIL(c, hipMemcpyAsync(c->raw_t, tt.data(), sizeof(double) * (j + 1),
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipMemcpyAsync(c->raw_r1, r1_host, sizeof(double) * (j + 1),
                                hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, igs::launch_update_raw(V, ldv, c->n, j, z, c->raw_t, c->raw_r1, inv_gamma,
                                        c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return IGS_OK;
}

static_assert(igs::kNoAllocMaxCols == IGS_NOALLOC_MAX_COLS, "no-allocation column limit");
static_assert(igs::kNoAllocBytes == (size_t)IGS_NOALLOC_BYTES, "no-allocation scratch size");

extern "C" int igs_kernel_reduce_noalloc(const double* V, int64_t ldv, int64_t n, int j,
                                         const double* z, double* PQ, void* hip_stream) {
  // every check before the first device call
  if (!V || !PQ) return set_err(nullptr, IGS_EINVAL, "V and PQ must be device pointers");
  if (n < 1 || ldv < n) return set_err(nullptr, IGS_EINVAL, "need n >= 1 and ldv >= n");
  if (j < 0 || j >= IGS_NOALLOC_MAX_COLS)
    return set_err(nullptr, IGS_EINVAL, "j = %d: the no-allocation reduction takes 0 <= j < %d",
                   j, IGS_NOALLOC_MAX_COLS);
  const hipError_t e = igs::launch_reduce_noalloc(V, ldv, n, j, z, PQ,
                                                  static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess)
    return set_err(nullptr, IGS_EDEVICE, "igs_kernel_reduce_noalloc: %s", hipGetErrorString(e));
  return IGS_OK;
}

extern "C" int igs_profile_get(igs_ctx* c, int which, int64_t* launches, double* total_ms,
                               double* total_bytes) {
  if (!c || which < 0 || which >= IGS_K_COUNT) return IGS_EINVAL;
  harvest(c, true);
  if (launches) *launches = c->stats[which].launches;
  if (total_ms) *total_ms = c->stats[which].ms;
  if (total_bytes) *total_bytes = c->stats[which].bytes;
  return IGS_OK;
}

extern "C" int igs_profile_reset(igs_ctx* c) {
  if (!c) return IGS_EINVAL;
  harvest(c, true);
  for (KStat& s : c->stats) s = KStat{};
  for (auto& row : c->stats_j)
    for (KStat& s : row) s = KStat{};
  return IGS_OK;
}

// ===========================================================================
// Autotuning of launch shapes
// ===========================================================================

extern "C" int igs_tune_reset(igs_ctx* c) {
  if (!c) return IGS_EINVAL;
  c->tune.clear();
  c->op.rpg = 0;
  c->tune_gen += 1;
  return IGS_OK;
}

extern "C" int igs_tune(igs_ctx* c, int restart, int gs_iters, igs_tune_report* rep) {
  if (!c) return IGS_EINVAL;
  c->err.clear();
  if (restart < 1 || (gs_iters != 1 && gs_iters != 2))
    return set_err(c, IGS_EINVAL, "restart >= 1 and gs_iters in {1, 2}");
  HIP_OR_FAIL(c, hipSetDevice(c->device));
  const long long n = c->n;
  const int m = (int)std::min<long long>(std::min<long long>(restart, n), IGS_MAX_RESTART);
  double* b = nullptr;
  double* x = nullptr;
  if (dalloc(&b, n) != hipSuccess || dalloc(&x, n) != hipSuccess) {
    if (b) (void)hipFree(b);
    return set_err(c, IGS_ENOMEM, "cannot allocate the tuning vectors");
  }
  {
    // a right-hand side with no special structure: b_i = 1 + (i mod 7) / 7
    std::vector<double> hb(n);
    for (long long i = 0; i < n; ++i) hb[i] = 1.0 + (double)(i % 7) / 7.0;
    if (hipMemcpy(b, hb.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(b);
      (void)hipFree(x);
      return set_err(c, IGS_EDEVICE, "cannot copy the tuning right-hand side");
    }
  }
  std::vector<double> red(m + 1), upd(m + 1);
  double total_ms = 0.0;
  // two full cycles (tol 0) with every launch timed; per-iteration totals
  auto measure = [&]() -> int {
    igs_profile_reset(c);
    HIP_OR_FAIL(c, hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
    igs_opts o{};
    o.profile = 1;
    o.max_cycles = 2;
    igs_info info{};
    const int rc = igs_solve_opts(c, b, x, restart, 0.0, gs_iters, &o, &info);
    if (rc < 0) return rc;
    harvest(c, true);
    total_ms = 0.0;
    for (int k = 0; k < IGS_K_COUNT; ++k) total_ms += c->stats[k].ms;
    for (int j = 0; j <= m; ++j) {
      red[j] = c->stats_j[IGS_K_REDUCE][j].ms + c->stats_j[IGS_K_OPREDUCE][j].ms;
      upd[j] = c->stats_j[IGS_K_UPDATE][j].ms;
    }
    return IGS_OK;
  };
  int rc = IGS_OK;
  igs_tune_reset(c);
  rc = measure();
  const double before = total_ms;
  const std::vector<double> red0 = red, upd0 = upd;
  int red_half = 0, upd_half = 0, best_rpg = 0;
  if (rc == IGS_OK) {
    // every iteration with half the blocks, then keep the halving where it
    // saved more than 3%
    c->tune.assign(IGS_MAX_RESTART + 1, 3);
    c->tune_gen += 1;
    rc = measure();
  }
  if (rc == IGS_OK) {
    std::vector<unsigned char> t(IGS_MAX_RESTART + 1, 0);
    for (int j = 0; j <= m; ++j) {
      if (red[j] > 0.0 && red[j] < 0.97 * red0[j]) { t[j] |= 1; ++red_half; }
      if (upd[j] > 0.0 && upd[j] < 0.97 * upd0[j]) { t[j] |= 2; ++upd_half; }
    }
    c->tune = t;
    c->tune_gen += 1;
    if (red_half + upd_half == 0) c->tune.clear();
  }
  if (rc == IGS_OK && !c->op.dense) {
    // rows per lane group of the operator apply
    const int lpr = c->op.lpr;
    const int cands[3] = {1, 2, 4};
    const int maxr = lpr <= 8 ? 4 : (lpr == 16 ? 2 : 1);
    // (compared on whole cycles: the default shape may run inside the
    // reduction's blocks, the others as a kernel of their own)
    c->op.rpg = 0;
    c->tune_gen += 1;
    rc = measure();
    double best = total_ms;
    for (int q = 0; q < 3 && rc == IGS_OK; ++q) {
      const int r = cands[q];
      if (r > maxr || r == (lpr <= 8 ? 4 : (lpr == 16 ? 2 : 1))) continue;   // the default
      c->op.rpg = r;
      c->tune_gen += 1;
      rc = measure();
      if (rc == IGS_OK && total_ms < 0.97 * best) {
        best = total_ms;
        best_rpg = r;
      }
    }
    c->op.rpg = best_rpg;
    c->tune_gen += 1;
  }
  double after = 0.0;
  if (rc == IGS_OK) {
    rc = measure();
    after = total_ms;
  }
  igs_profile_reset(c);
  (void)hipFree(b);
  (void)hipFree(x);
  if (rc != IGS_OK) {
    igs_tune_reset(c);
    return rc;
  }
  if (rep) {
    rep->cycle_ms_before = before / 2.0;
    rep->cycle_ms_after = after / 2.0;
    rep->spmv_rpg = best_rpg;
    rep->reduce_halved = red_half;
    rep->update_halved = upd_half;
    rep->reserved = 0;
  }
  return IGS_OK;
}

// ===========================================================================
// Serving: continuous batching of independent solves
// ===========================================================================

namespace {

// Device memory a request holds while it runs: its operator, b and x, and the
// basis and Hessenberg workspace of GMRES(m).
long long request_bytes(long long n, long long nnz, int m, bool fp32) {
  const long long mm = std::min<long long>(m, n);
  return 12 * nnz + 4 * (n + 1) + 8 * n * (mm + 5) + 32 * (mm + 2) * (mm + 2) +
         96 * n +   // the ELL form (at most 8 slots)
         (fp32 ? 4 * nnz + 4 * n * (mm + 2) + 32 * n : 0);
}

// A serving slot: a context with device capacity for CSR operators of up to
// n_cap rows and nnz_cap entries at restart m, plus b and x, on its own
// stream (or a shared one).  Requests are bound to it one at a time, so the
// serving loop allocates and frees no device memory (a free would wait for
// every stream).
struct Slot {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  igs_ctx* ctx = nullptr;
  double* b = nullptr;
  double* x = nullptr;
};

int slot_create(Slot& sl, long long n_cap, long long nnz_cap, int m, hipStream_t shared = nullptr,
                bool fp32 = false) {
  if (shared) {
    sl.stream = shared;
  } else {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
      return set_err(nullptr, IGS_EDEVICE, "cannot create a stream");
    sl.own_stream = true;
  }
  igs_ctx* c = nullptr;
  igs_ctx* out = nullptr;
  int rc = common_create(&out, sl.stream, &c);
  if (rc != IGS_OK) return rc;
  sl.ctx = c;
  c->n = n_cap;
  c->nnz = nnz_cap;
  c->n_cap = n_cap;
  c->nnz_cap = nnz_cap;
  if (dalloc(&c->d_row_ptr, n_cap + 1) != hipSuccess ||
      dalloc(&c->d_col, std::max<long long>(nnz_cap, 1)) != hipSuccess ||
      dalloc(&c->d_vals, std::max<long long>(nnz_cap, 1)) != hipSuccess ||
      dalloc(&sl.b, n_cap) != hipSuccess || dalloc(&sl.x, n_cap) != hipSuccess ||
      // the ELL form of operators with rows of at most 8 entries, built on
      // the device at each binding
      dalloc(&c->d_ell_col, 8 * n_cap) != hipSuccess ||
      dalloc(&c->d_ell_val, 8 * n_cap) != hipSuccess ||
      (fp32 && dalloc(&c->d_ell_val32, 8 * n_cap) != hipSuccess))
    return set_err(nullptr, IGS_ENOMEM, "device allocation of a serving slot failed");
  c->op.dense = 0;
  c->op.row_ptr = c->d_row_ptr;
  c->op.col_idx = c->d_col;
  c->op.vals = c->d_vals;
  const int mw = (int)std::min<long long>(m, std::min<long long>(n_cap, IGS_MAX_RESTART));
  rc = ensure_workspace(c, mw);
  if (rc == IGS_OK && fp32) {
    // the FP32 copy of the values is sized for the capacity; each binding
    // rounds the new operator into it
    if (hipMemsetAsync(c->d_vals, 0, sizeof(double) * std::max<long long>(nnz_cap, 1),
                       c->stream) != hipSuccess)
      return set_err(nullptr, IGS_EDEVICE, "cannot clear a serving slot");
    rc = ensure_fp32(c, mw);
  }
  if (rc != IGS_OK) return set_err(nullptr, rc, "%s", c->err.c_str());
  return IGS_OK;
}

void slot_destroy(Slot& sl) {
  if (sl.b) (void)hipFree(sl.b);
  if (sl.x) (void)hipFree(sl.x);
  if (sl.ctx) igs_destroy(sl.ctx);
  if (sl.stream && sl.own_stream) (void)hipStreamDestroy(sl.stream);
  sl = Slot{};
}

// Bind a host CSR operator to a slot (validated, copied on the slot's stream).
int slot_bind(igs_ctx* c, long long n, long long nnz, const int32_t* rp, const int32_t* ci,
              const double* va) {
  if (n < 1 || n > c->n_cap || nnz < 0 || nnz > c->nnz_cap || !rp || (nnz > 0 && (!ci || !va)))
    return set_err(c, IGS_EINVAL, "request of n = %lld, nnz = %lld exceeds the slot", n, nnz);
  const int rc = validate_csr(c, n, nnz, rp, ci, va);
  if (rc != IGS_OK) return rc;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_row_ptr, rp, sizeof(int32_t) * (n + 1),
                                hipMemcpyHostToDevice, c->stream));
  if (nnz > 0) {
    HIP_OR_FAIL(c, hipMemcpyAsync(c->d_col, ci, sizeof(int32_t) * nnz, hipMemcpyHostToDevice,
                                  c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->d_vals, va, sizeof(double) * nnz, hipMemcpyHostToDevice,
                                  c->stream));
  }
  const double avg = (double)nnz / (double)n;
  int lpr = 1;
  while (lpr < 64 && (double)lpr < avg) lpr *= 2;
  c->n = n;
  c->nnz = nnz;
  c->op.n = n;
  c->op.lpr = lpr;
  if (c->d_vals32) {   // FP32 values of the previous operator: round the new ones
    HIP_OR_FAIL(c, igs::launch_round_to_float(c->d_vals, c->d_vals32, nnz, c->stream));
  }
  // the ELL form, as igs_create keeps it (rows of at most 8 entries with 8
  // lanes per row), converted on the device from the copied CSR arrays
  long long kmax = 0;
  for (long long i = 0; i < n; ++i) kmax = std::max<long long>(kmax, rp[i + 1] - rp[i]);
  c->op.ell_k = 0;
  c->op.ell_col = nullptr;
  c->op.ell_val = nullptr;
  c->op.ell_val32 = nullptr;
  c->op.ell_dcol = nullptr;
  if (lpr == 8 && kmax >= 1 && kmax <= 8 && c->d_ell_col && c->d_ell_val) {
    HIP_OR_FAIL(c, igs::launch_csr_to_ell(n, (int)kmax, c->d_row_ptr, c->d_col, c->d_vals,
                                          c->d_ell_col, c->d_ell_val, c->stream));
    c->op.ell_k = (int)kmax;
    c->op.ell_col = c->d_ell_col;
    c->op.ell_val = c->d_ell_val;
    if (c->d_ell_val32) {
      HIP_OR_FAIL(c, igs::launch_round_to_float(c->d_ell_val, c->d_ell_val32, kmax * n,
                                                c->stream));
      c->op.ell_val32 = c->d_ell_val32;
    }
  }
  return IGS_OK;
}

}  // namespace

extern "C" int igs_serve(igs_request* reqs, int nreq, int slots, int64_t mem_cap, int restart,
                         double tol, int gs_iters, const igs_opts* opts, double* wall_seconds) {
  if (!reqs || nreq < 0 || slots < 1 || mem_cap <= 0 || restart < 1)
    return set_err(nullptr, IGS_EINVAL, "invalid serving arguments");
  if (nreq == 0) return IGS_OK;
  igs_opts o{};
  if (opts) o = *opts;
  o.keep_first_basis = 0;
  o.profile = 0;
  long long n_cap = 1, nnz_cap = 0;
  std::vector<long long> need(nreq);
  for (int i = 0; i < nreq; ++i) {
    reqs[i].rc = IGS_EINVAL;
    reqs[i].iters = 0;
    reqs[i].status = 0;
    reqs[i].t_admit = reqs[i].t_done = -1.0;
    if (reqs[i].n < 1 || reqs[i].nnz < 0 || !reqs[i].b || !reqs[i].x)
      return set_err(nullptr, IGS_EINVAL, "request %d: invalid size or NULL array", i);
    n_cap = std::max<long long>(n_cap, reqs[i].n);
    nnz_cap = std::max<long long>(nnz_cap, reqs[i].nnz);
    need[i] = request_bytes(reqs[i].n, reqs[i].nnz, restart, o.inner_fp32 != 0);
    if (need[i] > mem_cap)
      return set_err(nullptr, IGS_EINVAL, "request %d needs %lld bytes, more than the cap", i,
                     need[i]);
  }
  // Each slot holds the footprint of the largest request for the whole run:
  // run no more slots than the cap holds (at least one), so that the device
  // memory of the slots stays within it.
  const long long slot_bytes = request_bytes(n_cap, nnz_cap, restart, o.inner_fp32 != 0);
  slots = (int)std::max<long long>(1, std::min<long long>(slots, mem_cap / slot_bytes));
  std::vector<Slot> sl(slots);
  for (int k = 0; k < slots; ++k) {
    const int rc = slot_create(sl[k], n_cap, nnz_cap, restart, nullptr, o.inner_fp32 != 0);
    if (rc != IGS_OK) {
      for (Slot& x : sl) slot_destroy(x);
      return rc;
    }
  }
  std::vector<int> order(nreq);
  for (int i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival < reqs[b].arrival; });

  // Shared state: the FIFO of arrived requests and the device memory they hold.
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int> queue;
  long long reserved = 0;
  bool closed = false;
  const auto t0 = std::chrono::steady_clock::now();
  auto since = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  int device = 0;
  (void)hipGetDevice(&device);

  auto worker = [&](int k) {
    (void)hipSetDevice(device);
    Slot& me = sl[k];
    while (true) {
      int i = -1;
      {
        std::unique_lock<std::mutex> lk(mu);
        // admit the oldest arrived request once its memory fits the budget
        cv.wait(lk, [&] {
          return (!queue.empty() && reserved + need[queue.front()] <= mem_cap) ||
                 (closed && queue.empty());
        });
        if (queue.empty()) break;
        i = queue.front();
        queue.pop_front();
        reserved += need[i];
      }
      igs_request& r = reqs[i];
      r.t_admit = since();
      int rc = slot_bind(me.ctx, r.n, r.nnz, r.row_ptr, r.col_idx, r.vals);
      igs_info info{};
      if (rc == IGS_OK &&
          (hipMemcpyAsync(me.b, r.b, sizeof(double) * r.n, hipMemcpyHostToDevice, me.stream) !=
               hipSuccess ||
           hipMemsetAsync(me.x, 0, sizeof(double) * r.n, me.stream) != hipSuccess))
        rc = IGS_EDEVICE;
      if (rc == IGS_OK) rc = igs_solve_opts(me.ctx, me.b, me.x, restart, tol, gs_iters, &o, &info);
      if (rc == IGS_OK || rc == IGS_ENOCONV) {
        if (hipMemcpyAsync(r.x, me.x, sizeof(double) * r.n, hipMemcpyDeviceToHost, me.stream) !=
                hipSuccess ||
            hipStreamSynchronize(me.stream) != hipSuccess)
          rc = IGS_EDEVICE;
      }
      r.rc = rc;
      r.iters = info.iters;
      r.status = info.last_cycle_status;
      r.t_done = since();
      {
        std::lock_guard<std::mutex> lk(mu);
        reserved -= need[i];
      }
      cv.notify_all();
    }
  };
  std::vector<std::thread> threads;
  threads.reserve(slots);
  for (int k = 0; k < slots; ++k) threads.emplace_back(worker, k);
  // arrivals: each request joins the queue at its arrival time
  for (int idx = 0; idx < nreq; ++idx) {
    const int i = order[idx];
    const double at = reqs[i].arrival;
    std::this_thread::sleep_until(t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                           std::chrono::duration<double>(at > 0 ? at : 0.0)));
    {
      std::lock_guard<std::mutex> lk(mu);
      queue.push_back(i);
    }
    cv.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    closed = true;
  }
  cv.notify_all();
  for (std::thread& t : threads) t.join();
  if (wall_seconds) *wall_seconds = since();
  for (Slot& x : sl) slot_destroy(x);
  for (int i = 0; i < nreq; ++i)
    if (reqs[i].rc == IGS_EDEVICE) return IGS_EDEVICE;
  return IGS_OK;
}

// ===========================================================================
// Batches: many independent solves advanced by each launch
// ===========================================================================

namespace {

// One solve of a batch and where its restart loop stands (the same state
// machine as igs_solve_opts, advanced one cycle at a time).
struct Member {
  igs_ctx* c = nullptr;
  const double* b = nullptr;   // device
  double* x = nullptr;         // device
  int m = 0;                   // restart length min(restart, n)
  long long maxit = 0;
  long long its = 0;
  int cycles = 0;
  bool fresh = true;           // ||b|| not taken yet
  bool final_check = false;
  bool probe = false;          // this cycle is a check cycle after an Arnoldi-converged one
  bool skip_stagnation = false;
  bool done = false;
  bool converged = false;
  int rc = IGS_ENOCONV;
  int status = igs::kRunning;
  double bnorm = 0.0, relres = NAN, arn = NAN;
  double rho_prev = NAN;       // ||b - A x|| at the start of the previous cycle
  int breakdowns = 0, fallbacks = 0, J_first = -1, stagnant = 0;
};

struct Batch {
  hipStream_t stream = nullptr;
  igs::Inst* d_tab = nullptr;
  igs::Inst* h_tab = nullptr;   // pinned
  Ctl* d_ctl = nullptr;
  Ctl* h_ctl = nullptr;         // pinned
  Member mem[igs::kMaxBatch];
  std::string err;
};

struct BatchParams {
  int gs = 2;
  double tol = 0.0, tau = 1e-4, cycle_rtol = 0.0;
  int final_v = 0, fp32 = 0, max_cycles = 0;
  int reduce_rows = 2048, update_tiles = 1;
};

void batch_free(Batch& B) {
  if (B.d_tab) (void)hipFree(B.d_tab);
  if (B.d_ctl) (void)hipFree(B.d_ctl);
  if (B.h_tab) (void)hipHostFree(B.h_tab);
  if (B.h_ctl) (void)hipHostFree(B.h_ctl);
  B.d_tab = nullptr;
  B.d_ctl = nullptr;
  B.h_tab = nullptr;
  B.h_ctl = nullptr;
}

int batch_alloc(Batch& B, hipStream_t s) {
  B.stream = s;
  if (dalloc(&B.d_tab, igs::kMaxBatch) != hipSuccess || dalloc(&B.d_ctl, igs::kMaxBatch) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&B.h_tab), sizeof(igs::Inst) * igs::kMaxBatch,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&B.h_ctl), sizeof(Ctl) * igs::kMaxBatch,
                    hipHostMallocDefault) != hipSuccess) {
    batch_free(B);
    return IGS_ENOMEM;
  }
  memset(B.h_tab, 0, sizeof(igs::Inst) * igs::kMaxBatch);
  return IGS_OK;
}

// Put member k (context with workspace for its m, device b and x holding x0)
// into the batch.
void batch_add(Batch& B, int k, igs_ctx* c, const double* b, double* x, int restart,
               long long maxit_opt) {
  Member& M = B.mem[k];
  M = Member{};
  M.c = c;
  M.b = b;
  M.x = x;
  M.m = (int)std::min<long long>(std::min<long long>(restart, c->n), IGS_MAX_RESTART);
  M.maxit = maxit_opt > 0 ? maxit_opt : 20 * c->n;
}

#define BATCH_HIP(call)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      B.err = std::string(#call) + ": " + hipGetErrorString(e_);                               \
      return IGS_EDEVICE;                                                                      \
    }                                                                                          \
  } while (0)

// Fill row k of the host table from member k for the next cycle.
void batch_row(Batch& B, int k, const BatchParams& p) {
  const Member& M = B.mem[k];
  igs::Inst& I = B.h_tab[k];
  I.w = M.c->w;
  I.w.fp32 = p.fp32;
  I.w.pre_on = 0;   // batched updates form the small products themselves
  I.w.col_split = 0;
  I.op = M.c->op;
  I.n = M.c->n;
  I.b = M.b;
  I.x = M.x;
  I.its_before = M.its;
  const bool check = M.final_check || M.probe;
  I.maxit = check ? M.its : M.maxit;   // a check cycle runs iteration 0 only
  I.tol = p.tol;
  I.tau = p.tau;
  I.cycle_rtol = p.cycle_rtol;
  I.m = M.m;
  I.gs = p.gs;
  I.final_v = p.final_v;
  I.run_lsq = check ? 0 : 1;
}

// ||b|| and the finiteness of b and x0 for the members that just joined;
// a member with non-finite input leaves with IGS_EINVAL and x untouched.
int batch_admit(Batch& B, const BatchParams& p) {
  igs::BatchRun r{};
  r.d_tab = B.d_tab;
  r.h_tab = B.h_tab;
  r.stream = B.stream;
  r.reduce_rows = p.reduce_rows;
  r.update_tiles = p.update_tiles;
  for (int k = 0; k < igs::kMaxBatch; ++k) {
    Member& M = B.mem[k];
    if (!M.c || M.done || !M.fresh) continue;
    batch_row(B, k, p);
    r.act[r.count++] = k;
  }
  if (r.count == 0) return IGS_OK;
  BATCH_HIP(hipMemcpyAsync(B.d_tab, B.h_tab, sizeof(igs::Inst) * igs::kMaxBatch,
                           hipMemcpyHostToDevice, B.stream));
  BATCH_HIP(igs::batch_bnorm(r));
  BATCH_HIP(igs::batch_ctl_gather(r, B.d_ctl));
  BATCH_HIP(hipMemcpyAsync(B.h_ctl, B.d_ctl, sizeof(Ctl) * igs::kMaxBatch, hipMemcpyDeviceToHost,
                           B.stream));
  BATCH_HIP(hipStreamSynchronize(B.stream));
  for (int q = 0; q < r.count; ++q) {
    Member& M = B.mem[r.act[q]];
    const Ctl& h = B.h_ctl[r.act[q]];
    M.fresh = false;
    M.bnorm = h.bnorm;
    if (h.nonfinite_in > 0) {
      M.rc = IGS_EINVAL;
      M.done = true;
    }
  }
  return IGS_OK;
}

// One restart cycle of every member still running: the steps of
// igs_solve_opts, each launched once for all of them.
int batch_cycle(Batch& B, const BatchParams& p) {
  int rc = batch_admit(B, p);
  if (rc != IGS_OK) return rc;
  igs::BatchRun all{};
  all.d_tab = B.d_tab;
  all.h_tab = B.h_tab;
  all.stream = B.stream;
  all.reduce_rows = p.reduce_rows;
  all.update_tiles = p.update_tiles;
  int jmax = 0;
  for (int k = 0; k < igs::kMaxBatch; ++k) {
    Member& M = B.mem[k];
    if (!M.c || M.done) continue;
    batch_row(B, k, p);
    all.act[all.count++] = k;
    if (!M.final_check && !M.probe) jmax = std::max(jmax, M.m);
  }
  if (all.count == 0) return IGS_OK;
  BATCH_HIP(hipMemcpyAsync(B.d_tab, B.h_tab, sizeof(igs::Inst) * igs::kMaxBatch,
                           hipMemcpyHostToDevice, B.stream));
  BATCH_HIP(igs::batch_residual(all));
  // Iteration j runs for every member with j <= m (its tail step at j = m:
  // no operator apply, the reduction without z); the kernels of a member
  // whose cycle ended earlier return at once, as in a lone solve.
  int ng_full[igs::kMaxBatch];
  for (int j = 0; j <= jmax; ++j) {
    igs::BatchRun sp = all, rz = all, rt = all, up = all;
    sp.count = rz.count = rt.count = up.count = 0;
    for (int q = 0; q < all.count; ++q) {
      const int k = all.act[q];
      const Member& M = B.mem[k];
      const int mk = (M.final_check || M.probe) ? 0 : M.m;   // a check cycle stops after iteration 0
      if (j > mk) continue;
      up.act[up.count++] = k;
      if (j < M.m) {
        sp.act[sp.count++] = k;
        rz.act[rz.count++] = k;
      } else {
        rt.act[rt.count++] = k;
      }
    }
    if (up.count == 0) continue;
    BATCH_HIP(igs::batch_spmv(sp, j));
    int ngz[igs::kMaxBatch], ngt[igs::kMaxBatch];
    BATCH_HIP(igs::batch_reduce(rz, j, true, ngz));
    BATCH_HIP(igs::batch_reduce(rt, j, false, ngt));
    for (int q = 0; q < rz.count; ++q) ng_full[rz.act[q]] = ngz[q];
    for (int q = 0; q < rt.count; ++q) ng_full[rt.act[q]] = ngt[q];
    int ng[igs::kMaxBatch];
    for (int q = 0; q < up.count; ++q) ng[q] = ng_full[up.act[q]];
    BATCH_HIP(igs::batch_update(up, j, ng));
  }
  int mmax = 1;
  for (int q = 0; q < all.count; ++q) mmax = std::max(mmax, B.mem[all.act[q]].m);
  BATCH_HIP(igs::batch_lsq(all, mmax));
  BATCH_HIP(igs::batch_xupdate(all));
  BATCH_HIP(igs::batch_ctl_gather(all, B.d_ctl));
  BATCH_HIP(hipMemcpyAsync(B.h_ctl, B.d_ctl, sizeof(Ctl) * igs::kMaxBatch, hipMemcpyDeviceToHost,
                           B.stream));
  BATCH_HIP(hipStreamSynchronize(B.stream));
  for (int q = 0; q < all.count; ++q) {
    Member& M = B.mem[all.act[q]];
    const Ctl& h = B.h_ctl[all.act[q]];
    const int J = h.J;
    M.status = h.status;
    M.breakdowns = h.breakdowns;
    M.fallbacks = h.fallbacks;
    if (M.cycles == 0 && !M.final_check && !M.probe) M.J_first = J;
    M.cycles += 1;
    M.relres = M.bnorm > 0 ? h.rho / M.bnorm : h.rho;
    if (!M.skip_stagnation && cycle_stagnated(M.rho_prev, h.rho)) M.stagnant += 1;
    M.skip_stagnation = false;
    M.rho_prev = h.rho;
    if (M.status == igs::kConvStart) {
      M.converged = true;
      M.rc = IGS_OK;
      M.done = true;
    } else if (M.status == igs::kNonfinite) {
      M.rc = IGS_ENUMERIC;
      M.its += J;
      M.done = true;
    } else if (M.final_check) {
      M.rc = IGS_ENOCONV;
      M.done = true;
    } else if (M.probe) {
      // as in a lone solve: the true residual is above the tolerance, a
      // full cycle follows from the same x
      M.probe = false;
      M.skip_stagnation = true;
    } else {
      M.its += J;
      M.arn = M.bnorm > 0 ? h.gabs / M.bnorm : h.gabs;
      if (J == 0) {
        M.rc = IGS_ENUMERIC;
        M.done = true;
      } else if (M.its >= M.maxit || (p.max_cycles > 0 && M.cycles >= p.max_cycles)) {
        M.final_check = true;
      } else if (M.status == igs::kConverged && h.gabs <= h.tol_abs) {
        M.probe = true;
      }
    }
  }
  return IGS_OK;
}

#undef BATCH_HIP

void member_info(const Member& M, igs_info* info, double seconds) {
  if (!info) return;
  info->iters = M.its;
  info->cycles = M.cycles;
  info->relres_true = M.relres;
  info->arnoldi_relres = M.arn;
  info->bnorm = M.bnorm;
  info->converged = M.converged ? 1 : 0;
  info->breakdowns = M.breakdowns;
  info->lagnorm_fallbacks = M.fallbacks;
  info->last_cycle_status = M.status;
  info->first_cycle_J = M.J_first;
  info->stagnant_cycles = M.stagnant;
  info->seconds = seconds;
}

// Options a batch runs with (the subset of igs_solve_opts it supports).
int batch_params(const igs_opts& o, int gs_iters, double tol, BatchParams* p, std::string* why) {
  if (o.two_reduce) {
    *why = "the two-reduce comparator runs in igs_solve_opts only";
    return IGS_ENOTIMPL;
  }
  if (o.keep_first_basis) {
    *why = "keep_first_basis runs in igs_solve_opts only";
    return IGS_ENOTIMPL;
  }
  p->gs = gs_iters;
  p->tol = tol;
  p->tau = o.lagnorm_tau > 0.0 ? o.lagnorm_tau : 1e-4;
  p->final_v = o.final_basis_vector ? 1 : 0;
  p->fp32 = o.inner_fp32 ? 1 : 0;
  p->cycle_rtol = p->fp32 ? (o.inner_rtol > 0.0 ? o.inner_rtol : 1e-5) : 0.0;
  p->max_cycles = o.max_cycles;
  // defaults measured on the serving trace (128 requests): 2,048 rows and one
  // tile per block served 34.7 solves/s at 200 arrivals/s (33.1 with 4,096
  // rows and two tiles) and p50/p99 of 96/886 ms at 10/s (140/1,143)
  p->reduce_rows = o.batch_reduce_rows > 0 ? o.batch_reduce_rows : 2048;
  p->update_tiles = o.batch_update_tiles > 0 ? o.batch_update_tiles : 1;
  return IGS_OK;
}

}  // namespace

extern "C" int igs_solve_batch(igs_ctx* const* ctxs, const double* const* b, double* const* x,
                               int count, int restart, double tol, int gs_iters,
                               const igs_opts* opts, igs_info* infos, int* rcs) {
  if (!ctxs || !b || !x || count < 1 || count > IGS_MAX_BATCH || !ctxs[0])
    return set_err(nullptr, IGS_EINVAL, "invalid batch arguments (1 <= count <= %d)", IGS_MAX_BATCH);
  igs_ctx* c0 = ctxs[0];
  c0->err.clear();
  if (restart < 1) return set_err(c0, IGS_EINVAL, "restart must be >= 1");
  if (!(tol >= 0.0) || !isfinite(tol)) return set_err(c0, IGS_EINVAL, "tol must be finite, >= 0");
  if (gs_iters != 1 && gs_iters != 2) return set_err(c0, IGS_EINVAL, "gs_iters must be 1 or 2");
  igs_opts o{};
  if (opts) o = *opts;
  BatchParams p;
  std::string why;
  int rc = batch_params(o, gs_iters, tol, &p, &why);
  if (rc != IGS_OK) return set_err(c0, rc, "%s", why.c_str());
  const auto t0 = std::chrono::steady_clock::now();
  HIP_OR_FAIL(c0, hipSetDevice(c0->device));
  for (int k = 0; k < count; ++k) {
    igs_ctx* c = ctxs[k];
    if (!c || !b[k] || !x[k]) return set_err(c0, IGS_EINVAL, "member %d: NULL context or vector", k);
    if (c->device != c0->device) return set_err(c0, IGS_EINVAL, "member %d is on another device", k);
    if (c->op.dense) return set_err(c0, IGS_ENOTIMPL, "member %d: batches take CSR operators", k);
    if ((reinterpret_cast<uintptr_t>(b[k]) | reinterpret_cast<uintptr_t>(x[k])) % 16 != 0)
      return set_err(c0, IGS_EINVAL, "member %d: b and x must be 16-byte aligned", k);
    for (int q = 0; q < k; ++q)
      if (ctxs[q] == c) return set_err(c0, IGS_EINVAL, "member %d repeats a context", k);
  }
  for (int k = 0; k < count; ++k) {
    igs_ctx* c = ctxs[k];
    const int m = (int)std::min<long long>(std::min<long long>(restart, c->n), IGS_MAX_RESTART);
    rc = ensure_workspace(c, m);
    if (rc == IGS_OK && p.fp32) rc = ensure_fp32(c, m);
    if (rc != IGS_OK) return set_err(c0, rc, "member %d: %s", k, c->err.c_str());
    // work the caller queued on the member's own stream comes first
    HIP_OR_FAIL(c0, hipStreamSynchronize(c->stream));
  }
  Batch B;
  if (batch_alloc(B, c0->stream) != IGS_OK)
    return set_err(c0, IGS_ENOMEM, "cannot allocate the batch tables");
  for (int k = 0; k < count; ++k) batch_add(B, k, ctxs[k], b[k], x[k], restart, o.maxit);
  while (rc == IGS_OK) {
    bool running = false;
    for (int k = 0; k < count; ++k) running |= !B.mem[k].done;
    if (!running) break;
    rc = batch_cycle(B, p);
  }
  batch_free(B);
  if (rc != IGS_OK) return set_err(c0, rc, "%s", B.err.c_str());
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = IGS_OK;
  for (int k = 0; k < count; ++k) {
    member_info(B.mem[k], infos ? infos + k : nullptr, secs);
    if (rcs) rcs[k] = B.mem[k].rc;
    if (B.mem[k].rc < 0 && worst >= 0) worst = B.mem[k].rc;
    if (B.mem[k].rc == IGS_ENOCONV && worst == IGS_OK) worst = IGS_ENOCONV;
  }
  if (worst < 0) set_err(c0, worst, "a member of the batch failed (see its return code)");
  else if (worst == IGS_ENOCONV) set_err(c0, worst, "a member of the batch did not converge");
  return worst;
}

extern "C" int igs_serve_batched(igs_request* reqs, int nreq, int batch, int64_t mem_cap,
                                 int restart, double tol, int gs_iters, const igs_opts* opts,
                                 double* wall_seconds) {
  if (!reqs || nreq < 0 || batch < 1 || batch > IGS_MAX_BATCH || mem_cap <= 0 || restart < 1)
    return set_err(nullptr, IGS_EINVAL, "invalid serving arguments (1 <= batch <= %d)",
                   IGS_MAX_BATCH);
  if (!(tol >= 0.0) || !isfinite(tol) || (gs_iters != 1 && gs_iters != 2))
    return set_err(nullptr, IGS_EINVAL, "invalid tol or gs_iters");
  if (nreq == 0) return IGS_OK;
  igs_opts o{};
  if (opts) o = *opts;
  o.keep_first_basis = 0;
  o.profile = 0;
  BatchParams p;
  std::string why;
  int rc = batch_params(o, gs_iters, tol, &p, &why);
  if (rc != IGS_OK) return set_err(nullptr, rc, "%s", why.c_str());
  long long n_cap = 1, nnz_cap = 0;
  std::vector<long long> need(nreq);
  for (int i = 0; i < nreq; ++i) {
    reqs[i].rc = IGS_EINVAL;
    reqs[i].iters = 0;
    reqs[i].status = 0;
    reqs[i].t_admit = reqs[i].t_done = -1.0;
    if (reqs[i].n < 1 || reqs[i].nnz < 0 || !reqs[i].b || !reqs[i].x)
      return set_err(nullptr, IGS_EINVAL, "request %d: invalid size or NULL array", i);
    n_cap = std::max<long long>(n_cap, reqs[i].n);
    nnz_cap = std::max<long long>(nnz_cap, reqs[i].nnz);
    need[i] = request_bytes(reqs[i].n, reqs[i].nnz, restart, p.fp32 != 0);
    if (need[i] > mem_cap)
      return set_err(nullptr, IGS_EINVAL, "request %d needs %lld bytes, more than the cap", i,
                     need[i]);
  }
  // as igs_serve: no more members than the cap holds at the largest footprint
  const long long slot_bytes = request_bytes(n_cap, nnz_cap, restart, p.fp32 != 0);
  batch = (int)std::max<long long>(1, std::min<long long>(batch, mem_cap / slot_bytes));
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
    return set_err(nullptr, IGS_EDEVICE, "cannot create a stream");
  std::vector<Slot> sl(batch);
  Batch B;
  rc = batch_alloc(B, stream) == IGS_OK ? IGS_OK : set_err(nullptr, IGS_ENOMEM, "batch tables");
  for (int k = 0; k < batch && rc == IGS_OK; ++k)
    rc = slot_create(sl[k], n_cap, nnz_cap, restart, stream, p.fp32 != 0);
  auto cleanup = [&]() {
    for (Slot& x : sl) slot_destroy(x);
    batch_free(B);
    (void)hipStreamDestroy(stream);
  };
  if (rc != IGS_OK) {
    cleanup();
    return rc;
  }
  std::vector<int> order(nreq);
  for (int i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival < reqs[b].arrival; });
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int> queue;
  bool closed = false;
  bool stop = false;   // the loop ended early: arrivals stop too
  const auto t0 = std::chrono::steady_clock::now();
  auto since = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  // arrivals: each request joins the queue at its arrival time
  std::thread arrivals([&]() {
    for (int idx = 0; idx < nreq; ++idx) {
      const int i = order[idx];
      const double at = reqs[i].arrival;
      const auto when = t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                 std::chrono::duration<double>(at > 0 ? at : 0.0));
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait_until(lk, when, [&] { return stop; });
        if (stop) break;
        queue.push_back(i);
      }
      cv.notify_all();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      closed = true;
    }
    cv.notify_all();
  });
  std::vector<int> req_of(batch, -1);
  long long reserved = 0;
  int fatal = IGS_OK;
  while (fatal == IGS_OK) {
    // admit: the oldest arrived requests, while a member is free and the
    // memory they hold fits the cap
    std::vector<int> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      bool any = false;
      for (int k = 0; k < batch; ++k) any |= (req_of[k] >= 0);
      if (!any)
        cv.wait(lk, [&] { return !queue.empty() || closed; });
      for (int k = 0; k < batch && !queue.empty(); ++k) {
        if (req_of[k] >= 0) continue;
        const int i = queue.front();
        if (reserved + need[i] > mem_cap) break;
        queue.pop_front();
        reserved += need[i];
        req_of[k] = i;
        admitted.push_back(k);
      }
      if (!any && admitted.empty() && closed && queue.empty()) break;
    }
    for (int k : admitted) {
      igs_request& r = reqs[req_of[k]];
      r.t_admit = since();
      igs_ctx* c = sl[k].ctx;
      int brc = slot_bind(c, r.n, r.nnz, r.row_ptr, r.col_idx, r.vals);
      if (brc == IGS_OK &&
          (hipMemcpyAsync(sl[k].b, r.b, sizeof(double) * r.n, hipMemcpyHostToDevice, stream) !=
               hipSuccess ||
           hipMemsetAsync(sl[k].x, 0, sizeof(double) * r.n, stream) != hipSuccess))
        brc = IGS_EDEVICE;
      if (brc != IGS_OK) {
        r.rc = brc;
        r.t_done = since();
        reserved -= need[req_of[k]];
        req_of[k] = -1;
        B.mem[k] = Member{};
        if (brc == IGS_EDEVICE) fatal = brc;
        continue;
      }
      batch_add(B, k, c, sl[k].b, sl[k].x, restart, o.maxit);
    }
    if (fatal != IGS_OK) break;
    bool running = false;
    for (int k = 0; k < batch; ++k) running |= (req_of[k] >= 0);
    if (!running) continue;
    rc = batch_cycle(B, p);
    if (rc != IGS_OK) {
      fatal = rc;
      break;
    }
    // completions: copy x back, free the member and its memory
    bool copied = false;
    for (int k = 0; k < batch; ++k) {
      if (req_of[k] < 0 || !B.mem[k].done) continue;
      igs_request& r = reqs[req_of[k]];
      if (B.mem[k].rc == IGS_OK || B.mem[k].rc == IGS_ENOCONV || B.mem[k].rc == IGS_ENUMERIC) {
        if (hipMemcpyAsync(r.x, sl[k].x, sizeof(double) * r.n, hipMemcpyDeviceToHost, stream) !=
            hipSuccess)
          fatal = IGS_EDEVICE;
        copied = true;
      }
    }
    if (copied && hipStreamSynchronize(stream) != hipSuccess) fatal = IGS_EDEVICE;
    for (int k = 0; k < batch; ++k) {
      if (req_of[k] < 0 || !B.mem[k].done) continue;
      igs_request& r = reqs[req_of[k]];
      r.rc = B.mem[k].rc;
      r.iters = B.mem[k].its;
      r.status = B.mem[k].status;
      r.t_done = since();
      reserved -= need[req_of[k]];
      req_of[k] = -1;
      B.mem[k] = Member{};
    }
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv.notify_all();
  arrivals.join();
  if (wall_seconds) *wall_seconds = since();
  const std::string why_fatal = B.err;
  cleanup();
  if (fatal != IGS_OK) return set_err(nullptr, fatal, "serving stopped: %s", why_fatal.c_str());
  return IGS_OK;
}
