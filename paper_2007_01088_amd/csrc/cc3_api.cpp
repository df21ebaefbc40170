// C ABI of libcc3 (declared in include/cc3.h): argument checks, the workspace
// plan, and the launch sequence of one residual evaluation (Algorithm 1):
// T1 transformation and integral-block build, the batched triple loop, the
// covariant back-transformation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cc3.h"
#include "cc3_internal.hpp"

using namespace cc3;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(CC3_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

extern "C" const char* cc3_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// context and kernel timing
// ---------------------------------------------------------------------------
struct TimedLaunch {
  int family;
  hipEvent_t start, stop;
  double flops, bytes;
};

static const char* kFamilies[] = {"t1_transform", "block_build",  "w_build",
                                  "mix",          "omega_contract", "reduce", "back_transform"};
enum { FAM_T1 = 0, FAM_BUILD, FAM_W, FAM_MIX, FAM_OMEGA, FAM_REDUCE, FAM_BACK, NFAM };

// The triple loop alternates its batches between two internal streams (each
// with its own cube and slab buffers), so that one batch's W build and mix
// overlap the previous batch's Omega contraction; the reductions into the
// residual are chained by events in batch order.
enum { NSTREAM = 2 };

struct cc3_ctx {
  int device;
  bool profiling = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> pool;
  std::mutex mu;
  bool have_streams = false;
  hipStream_t s[NSTREAM];
  hipEvent_t ev_fork, ev_done[NSTREAM], ev_red[NSTREAM];
};

static int ensure_streams(cc3_ctx* c) {
  if (c->have_streams) return CC3_OK;
  for (int k = 0; k < NSTREAM; ++k) {
    if (hipStreamCreateWithFlags(&c->s[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_done[k], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_red[k], hipEventDisableTiming) != hipSuccess)
      return fail(CC3_E_DEVICE, "could not create the internal streams");
  }
  if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess)
    return fail(CC3_E_DEVICE, "could not create the internal streams");
  c->have_streams = true;
  return CC3_OK;
}

static hipEvent_t take_event(cc3_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when profiling is on.
struct Timer {
  cc3_ctx* c;
  hipStream_t st;
  TimedLaunch tl;
  bool on;
  Timer(cc3_ctx* c_, hipStream_t st_, int fam, double flops, double bytes) : c(c_), st(st_) {
    on = c->profiling;
    if (!on) return;
    tl.family = fam;
    tl.flops = flops;
    tl.bytes = bytes;
    tl.start = take_event(c);
    tl.stop = take_event(c);
    if (!tl.start || !tl.stop) { on = false; return; }
    hipEventRecord(tl.start, st);
  }
  ~Timer() {
    if (!on) return;
    hipEventRecord(tl.stop, st);
    c->timed.push_back(tl);
  }
};

extern "C" int cc3_create(cc3_ctx** out, int device) {
  if (!out) return fail(CC3_E_INVAL, "cc3_create: out is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n)
    return fail(CC3_E_INVAL, "cc3_create: device %d out of range (%d devices)", device, n);
  cc3_ctx* c = new cc3_ctx();
  c->device = device;
  *out = c;
  return CC3_OK;
}

extern "C" int cc3_destroy(cc3_ctx* c) {
  if (!c) return CC3_OK;
  for (auto& t : c->timed) { hipEventDestroy(t.start); hipEventDestroy(t.stop); }
  for (auto e : c->pool) hipEventDestroy(e);
  if (c->have_streams) {
    for (int k = 0; k < NSTREAM; ++k) {
      hipStreamDestroy(c->s[k]);
      hipEventDestroy(c->ev_done[k]);
      hipEventDestroy(c->ev_red[k]);
    }
    hipEventDestroy(c->ev_fork);
  }
  delete c;
  return CC3_OK;
}

extern "C" int cc3_profile_enable(cc3_ctx* c, int on) {
  if (!c) return fail(CC3_E_INVAL, "cc3_profile_enable: ctx is NULL");
  std::lock_guard<std::mutex> g(c->mu);
  for (auto& t : c->timed) { c->pool.push_back(t.start); c->pool.push_back(t.stop); }
  c->timed.clear();
  c->profiling = on != 0;
  return CC3_OK;
}

extern "C" int cc3_profile_get(cc3_ctx* c, cc3_kernel_stat* out, int max, int* count) {
  if (!c || !out || !count || max < 0) return fail(CC3_E_INVAL, "cc3_profile_get: bad argument");
  std::lock_guard<std::mutex> g(c->mu);
  cc3_kernel_stat st[NFAM];
  memset(st, 0, sizeof st);
  for (int f = 0; f < NFAM; ++f) snprintf(st[f].name, sizeof st[f].name, "%s", kFamilies[f]);
  for (auto& t : c->timed) {
    HIPCHK(hipEventSynchronize(t.stop));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t.start, t.stop));
    st[t.family].launches += 1;
    st[t.family].total_ms += ms;
    st[t.family].flops += t.flops;
    st[t.family].bytes += t.bytes;
  }
  int n = 0;
  for (int f = 0; f < NFAM && n < max; ++f)
    if (st[f].launches > 0) out[n++] = st[f];
  *count = n;
  return CC3_OK;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int env_int(const char* name, int dflt) {
  const char* s = getenv(name);
  if (!s || !*s) return dflt;
  int v = atoi(s);
  return v > 0 ? v : dflt;
}

namespace cc3 {

int make_plan(int no, int nv, int nchol, int prec, unsigned flags, Plan* p, int batch_override) {
  memset(p, 0, sizeof *p);
  p->no = no; p->nv = nv; p->nchol = nchol; p->prec = prec; p->flags = flags;
  const size_t o = no, v = nv, J = nchol;
  p->ntri = (int)((size_t)no * (no + 1) * (no + 2) / 6 - no);
  p->cube = v * v * v;
  // triples per batch: enough W-build workgroups per launch to fill 256 CUs
  // many times over, bounded by a cube-memory budget
  const size_t wg_per_triple = 3 * v * ((v + 127) / 128) * ((v + 127) / 128);
  int batch = (int)std::max<size_t>(1, (size_t)(12288 + wg_per_triple - 1) / wg_per_triple);
  const size_t budget = (size_t)env_int("CC3_CUBE_BUDGET_MB", 4096) << 20;
  const size_t per_triple = 5 * p->cube * sizeof(double);
  batch = (int)std::min<size_t>((size_t)batch, std::max<size_t>(1, budget / per_triple));
  batch = env_int("CC3_BATCH", batch);
  if (batch_override > 0) batch = batch_override;
  batch = std::min(batch, 160);  // the reduction lists at most 6 * 160 pairs per p
  batch = std::max(1, std::min(batch, std::max(1, p->ntri)));
  p->batch = batch;
  // largest (triples x chunks) product over the batch sizes the loop can see
  size_t tc = 1;
  for (int nb = 1; nb <= batch; ++nb) tc = std::max(tc, (size_t)nb * omega_nbchunks(nv, nb));
  p->pvv_entries = tc;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
  p->off_Gw = take(o * v * v * v * 8);
  p->off_Gv = take(o * v * v * v * 8);
  p->off_Go = take(o * o * o * v * 8);
  p->off_Jo = take(o * o * v * v * 8);
  p->off_Hs = take(o * o * o * v * 8);
  p->off_F = take(o * v * 8);
  p->off_Ot1 = take(o * v * 8);
  p->off_Ot2 = take(o * o * v * v * 8);
  p->off_OtT = take(o * o * v * v * 8);
  p->off_t2N = take(o * o * v * v * 8);
  p->off_lp = take(lp_operand_bytes(prec, no, nv));
  p->pvv_bytes = align256(tc * 6 * v * (v + 1) * 8);
  p->soo_bytes = align256((size_t)batch * 6 * o * v * v * 8);
  p->off_Pvv = take(2 * p->pvv_bytes);
  p->off_Soo = take(2 * p->soo_bytes);
  p->off_tri = take((size_t)std::max(1, p->ntri) * 3 * sizeof(int) + 64);
  p->off_flag = take(64);
  // the Cholesky scratch is dead once the blocks are built: it shares the cube region
  p->chol_bytes = J ? align256(J * v * v * 8) * 2 + align256(J * o * o * 8) * 2 +
                          align256(J * o * v * 8) * 2 + align256(J * 8) + align256(J * o * o * 8)
                    : 0;
  p->cube_bytes = align256((size_t)batch * 5 * p->cube * 8);
  p->off_cubes = take(std::max(p->chol_bytes, 2 * p->cube_bytes));
  p->off_chol = p->off_cubes;
  p->total = off;
  return CC3_OK;
}

}  // namespace cc3

static int check_sizes(int no, int nv, int nchol, int prec) {
  if (no < 1 || nv < 1) return fail(CC3_E_INVAL, "sizes must be positive (no=%d nv=%d)", no, nv);
  if (nchol < 0) return fail(CC3_E_INVAL, "nchol must be >= 0 (got %d)", nchol);
  if (no > 63 || nv > 1024)
    return fail(CC3_E_INVAL, "sizes beyond the supported range no <= 63, nv <= 1024 (no=%d nv=%d)",
                no, nv);
  if (prec != CC3_FP64 && prec != CC3_FP32 && prec != CC3_BF16X3 && prec != CC3_BF16X6)
    return fail(CC3_E_INVAL, "unknown precision %d", prec);
  return CC3_OK;
}

extern "C" int cc3_workspace_size(int no, int nv, int nchol, int prec, unsigned flags,
                                  size_t* bytes) {
  if (!bytes) return fail(CC3_E_INVAL, "cc3_workspace_size: bytes is NULL");
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  Plan p;
  make_plan(no, nv, nchol, prec, flags, &p, 0);
  *bytes = p.total;
  return CC3_OK;
}

extern "C" int cc3_flops(int no, int nv, double* nominal, double* executed) {
  if (no < 1 || nv < 1) return fail(CC3_E_INVAL, "cc3_flops: sizes must be positive");
  const double v = nv, o = no;
  if (nominal) *nominal = 4.0 * v * v * v * v * o * o * o;
  if (executed) {
    const double D = o * (o - 1) * (o - 2) / 6.0, E = o * (o - 1);
    const double w = 2.0 * v * v * v * v + 2.0 * v * v * v * o;
    const double perm = 2.0 * v * v * v * v + 2.0 * v * v * v * (o + 2.0);
    *executed = (6.0 * D + 3.0 * E) * (w + perm);
  }
  return CC3_OK;
}

static int check_dev_ptr(const void* p, const char* what) {
  if (!p) return fail(CC3_E_INVAL, "%s is NULL", what);
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CC3_E_INVAL, "%s is not device memory", what);
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(CC3_E_INVAL, "%s is not device memory", what);
  return CC3_OK;
}

// ---------------------------------------------------------------------------
// the residual
// ---------------------------------------------------------------------------
struct Ws {
  Blocks b;
  CholeskyScratch cs;
  double *Ot1, *Ot2, *OtT, *t2N;
  double *cubes[2], *Pvv[2], *Soo[2];
  int* tri;
  int* flag;
  LpOperands lp;
};

static Ws carve(const Plan& p, void* ws) {
  char* base = (char*)ws;
  Ws w;
  w.b.Gw = (double*)(base + p.off_Gw);
  w.b.Gv = (double*)(base + p.off_Gv);
  w.b.Go = (double*)(base + p.off_Go);
  w.b.Jo = (double*)(base + p.off_Jo);
  w.b.Hs = (double*)(base + p.off_Hs);
  w.b.F = (double*)(base + p.off_F);
  w.Ot1 = (double*)(base + p.off_Ot1);
  w.Ot2 = (double*)(base + p.off_Ot2);
  w.OtT = (double*)(base + p.off_OtT);
  w.t2N = (double*)(base + p.off_t2N);
  lp_operand_ptrs(p.prec, p.no, p.nv, base + p.off_lp, w.lp);
  for (int k = 0; k < 2; ++k) {
    w.Pvv[k] = (double*)(base + p.off_Pvv + k * p.pvv_bytes);
    w.Soo[k] = (double*)(base + p.off_Soo + k * p.soo_bytes);
    w.cubes[k] = (double*)(base + p.off_cubes + k * p.cube_bytes);
  }
  w.tri = (int*)(base + p.off_tri);
  w.flag = (int*)(base + p.off_flag);
  const size_t J = p.nchol, o = p.no, v = p.nv;
  char* c = base + p.off_chol;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* at = c + off; off = align256(off + bytes); return (double*)at; };
  w.cs.Lvv = take(J * v * v * 8);
  w.cs.LvvT = take(J * v * v * 8);
  w.cs.Loo = take(J * o * o * 8);
  w.cs.LooT = take(J * o * o * 8);
  w.cs.LvoT = take(J * o * v * 8);
  w.cs.Lov = take(J * o * v * 8);
  w.cs.s = take(J * 8);
  w.cs.M = take(J * o * o * 8);
  return w;
}

static void host_triples(int no, std::vector<int>& t) {
  t.clear();
  for (int i = 0; i < no; ++i)
    for (int j = 0; j <= i; ++j)
      for (int k = 0; k <= j; ++k)
        if (!(i == j && j == k)) { t.push_back(i); t.push_back(j); t.push_back(k); }
}

static int kind_of(int i, int j, int k) { return (i == j) ? 1 : (j == k) ? 2 : 0; }

// The batched triple loop over a device triple table `tri` of n entries whose
// host copy is `ht` (for FLOP accounting only).  Batch b runs on internal
// stream b % 2 with buffer set b % 2; reduction b waits for reduction b - 1.
static int triple_loop(cc3_ctx* c, const Plan& p, const Ws& w, const double* eps, const double* t2,
                       const int* tri, const int* ht, int n, hipStream_t st) {
  int rc = ensure_streams(c);
  if (rc) return rc;
  std::vector<int> kinds;
  launch_t2N(t2, w.t2N, p.no, p.nv, st);
  if (p.prec != CC3_FP64) launch_lp_convert(t2, w.b, p.no, p.nv, w.lp, st);
  HIPCHK(hipEventRecord(c->ev_fork, st));
  for (int k = 0; k < NSTREAM; ++k) HIPCHK(hipStreamWaitEvent(c->s[k], c->ev_fork, 0));
  int nbatch = 0;
  for (int t0 = 0; t0 < n; t0 += p.batch, ++nbatch) {
    const int nb = std::min(p.batch, n - t0);
    const int k = nbatch % NSTREAM;
    hipStream_t sk = c->s[k];
    kinds.resize(nb);
    for (int t = 0; t < nb; ++t)
      kinds[t] = kind_of(ht[3 * (t0 + t)], ht[3 * (t0 + t) + 1], ht[3 * (t0 + t) + 2]);
    const int* tb = tri + 3 * t0;
    {
      Timer tm(c, sk, FAM_W, wbuild_flops(p.no, p.nv, kinds.data(), nb), 0.0);
      if (p.prec == CC3_FP64)
        launch_wbuild(t2, w.t2N, w.b, tb, nb, w.cubes[k], p.no, p.nv, false, sk);
      else
        launch_wbuild_lp(w.lp, tb, nb, w.cubes[k], p.no, p.nv, false, sk);
    }
    {
      Timer tm(c, sk, FAM_MIX, 0.0, 0.0);
      launch_mix(eps, tb, nb, w.cubes[k], p.no, p.nv, sk);
    }
    {
      Timer tm(c, sk, FAM_OMEGA, omega_flops(p.no, p.nv, kinds.data(), nb), 0.0);
      launch_omega(w.cubes[k], w.b, tb, nb, w.Pvv[k], w.Soo[k], p.no, p.nv, sk);
    }
    if (nbatch > 0) HIPCHK(hipStreamWaitEvent(sk, c->ev_red[(nbatch - 1) % NSTREAM], 0));
    {
      Timer tm(c, sk, FAM_REDUCE, 0.0, 0.0);
      launch_reduce(tb, nb, w.Pvv[k], w.Soo[k], w.Ot1, w.Ot2, w.OtT, p.no, p.nv, sk);
    }
    HIPCHK(hipEventRecord(c->ev_red[k], sk));
  }
  for (int k = 0; k < NSTREAM; ++k) {
    HIPCHK(hipEventRecord(c->ev_done[k], c->s[k]));
    HIPCHK(hipStreamWaitEvent(st, c->ev_done[k], 0));
  }
  return CC3_OK;
}

static int prepare_cholesky(cc3_ctx* c, const Plan& p, const Ws& w, const double* L,
                            const double* t1, hipStream_t st) {
  {
    Timer tm(c, st, FAM_T1, 0.0, 0.0);
    launch_t1_transform(L, t1, w.cs, p.no, p.nv, p.nchol, st);
    launch_fock(t1, w.cs, w.b.F, p.no, p.nv, p.nchol, st);
  }
  {
    const double v = p.nv, o = p.no, J = p.nchol;
    const double fl = 2.0 * J * (2.0 * v * v * v * o + o * o * v * v + 2.0 * o * o * o * v);
    Timer tm(c, st, FAM_BUILD, fl, 0.0);
    launch_build_blocks(w.cs, w.b, p.no, p.nv, p.nchol, st);
  }
  return CC3_OK;
}

// CC3_CHECK: blocks the host until the input check has run.
static int run_input_check(const Plan& p, const Ws& w, const double* eps, const double* L,
                           const double* t2, hipStream_t st) {
  launch_check(eps, L, t2, p.no, p.nv, p.nchol, w.flag, st);
  int bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, w.flag, sizeof bits, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (bits & 1) return fail(CC3_E_PRECOND, "t2 violates t2[i][j][a][b] == t2[j][i][b][a]");
  if (bits & 2) return fail(CC3_E_PRECOND, "L violates L[J][p][q] == L[J][q][p]");
  if (bits & 4) return fail(CC3_E_PRECOND, "a denominator eps^{abc}_{ijk} is not positive");
  return CC3_OK;
}

static int common_checks(cc3_ctx* c, int no, int nv, int nchol, int prec, unsigned flags,
                         void* ws, size_t ws_bytes, Plan* p) {
  if (!c) return fail(CC3_E_INVAL, "ctx is NULL");
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  if (flags & ~(unsigned)(CC3_ACCUMULATE | CC3_CHECK))
    return fail(CC3_E_INVAL, "unknown flag bits 0x%x", flags);
  make_plan(no, nv, nchol, prec, flags, p, 0);
  if (!ws) return fail(CC3_E_INVAL, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return fail(CC3_E_INVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < p->total)
    return fail(CC3_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, p->total);
  HIPCHK(hipSetDevice(c->device));
  return check_dev_ptr(ws, "workspace");
}

extern "C" int cc3_triples_residual(cc3_ctx* c, int no, int nv, int nchol, const double* eps,
                                    const double* L, const double* t1, const double* t2,
                                    double* omega1, double* omega2, int prec, unsigned flags,
                                    void* ws, size_t ws_bytes, cc3_stream_t stream) {
  Plan p;
  int rc = common_checks(c, no, nv, nchol, prec, flags, ws, ws_bytes, &p);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1 for the Cholesky form");
  const void* ptrs[] = {eps, L, t1, t2, omega1, omega2};
  const char* names[] = {"eps", "L", "t1", "t2", "omega1", "omega2"};
  for (int i = 0; i < 6; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  prepare_cholesky(c, p, w, L, t1, st);
  launch_fill(w.Ot1, (int64_t)no * nv, 0.0, st);
  launch_fill(w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
  launch_fill(w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
  launch_triple_table(w.tri, no, st);
  std::vector<int> ht;
  host_triples(no, ht);
  if ((rc = triple_loop(c, p, w, eps, t2, w.tri, ht.data(), p.ntri, st))) return rc;
  {
    Timer tm(c, st, FAM_BACK, 0.0, 0.0);
    launch_back_transform(w.Ot1, w.Ot2, w.OtT, omega1, omega2, no, nv,
                          (flags & CC3_ACCUMULATE) != 0, st);
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

extern "C" int cc3_triples_residual_blocks(cc3_ctx* c, int no, int nv, const double* eps,
                                           const double* g_vvvo, const double* g_oovo,
                                           const double* g_ovov, const double* g_ooov,
                                           const double* g_vvov, const double* F_ov,
                                           const double* t2, double* omega1, double* omega2,
                                           int prec, unsigned flags, void* ws, size_t ws_bytes,
                                           cc3_stream_t stream) {
  Plan p;
  int rc = common_checks(c, no, nv, 0, prec, flags, ws, ws_bytes, &p);
  if (rc) return rc;
  const void* ptrs[] = {eps, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, t2, omega1, omega2};
  const char* names[] = {"eps", "g_vvvo", "g_oovo", "g_ovov", "g_ooov",
                         "g_vvov", "F_ov", "t2", "omega1", "omega2"};
  for (int i = 0; i < 10; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, nullptr, t2, st))) return rc;
  {
    Timer tm(c, st, FAM_BUILD, 0.0, 0.0);
    launch_relayout_blocks(g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, w.b, no, nv, st);
  }
  launch_fill(w.Ot1, (int64_t)no * nv, 0.0, st);
  launch_fill(w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
  launch_fill(w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
  launch_triple_table(w.tri, no, st);
  std::vector<int> ht;
  host_triples(no, ht);
  if ((rc = triple_loop(c, p, w, eps, t2, w.tri, ht.data(), p.ntri, st))) return rc;
  {
    Timer tm(c, st, FAM_BACK, 0.0, 0.0);
    launch_back_transform(w.Ot1, w.Ot2, w.OtT, omega1, omega2, no, nv,
                          (flags & CC3_ACCUMULATE) != 0, st);
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

extern "C" int cc3_triples_residual_subset(cc3_ctx* c, int no, int nv, int nchol,
                                           const double* eps, const double* L, const double* t1,
                                           const double* t2, const int32_t* triples, int ntriples,
                                           double* omega1_tilde, double* omega2_tilde, int prec,
                                           unsigned flags, void* ws, size_t ws_bytes,
                                           cc3_stream_t stream) {
  Plan p;
  int rc = common_checks(c, no, nv, nchol, prec, flags, ws, ws_bytes, &p);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1 for the Cholesky form");
  if (ntriples < 0 || ntriples > p.ntri)
    return fail(CC3_E_INVAL, "ntriples %d out of range [0, %d]", ntriples, p.ntri);
  if (ntriples > 0 && !triples) return fail(CC3_E_INVAL, "triples is NULL");
  for (int t = 0; t < ntriples; ++t) {
    const int i = triples[3 * t], j = triples[3 * t + 1], k = triples[3 * t + 2];
    if (!(i < no && i >= j && j >= k && k >= 0) || (i == j && j == k))
      return fail(CC3_E_INVAL, "triple %d = (%d,%d,%d) is not an unordered triple i>=j>=k "
                  "(not all equal) below no=%d", t, i, j, k, no);
  }
  const void* ptrs[] = {eps, L, t1, t2, omega1_tilde, omega2_tilde};
  const char* names[] = {"eps", "L", "t1", "t2", "omega1_tilde", "omega2_tilde"};
  for (int i = 0; i < 6; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  prepare_cholesky(c, p, w, L, t1, st);
  launch_fill(w.Ot1, (int64_t)no * nv, 0.0, st);
  launch_fill(w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
  launch_fill(w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
  if (ntriples > 0) {
    HIPCHK(hipMemcpyAsync(w.tri, triples, sizeof(int) * 3 * (size_t)ntriples,
                          hipMemcpyHostToDevice, st));
    if ((rc = triple_loop(c, p, w, eps, t2, w.tri, triples, ntriples, st))) return rc;
  }
  launch_combine(w.Ot1, w.Ot2, w.OtT, omega1_tilde, omega2_tilde, no, nv, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return CC3_OK;
}

extern "C" int cc3_t3_block(cc3_ctx* c, int no, int nv, int nchol, const double* eps,
                            const double* L, const double* t1, const double* t2, int i, int j,
                            int k, double* tau, int prec, void* ws, size_t ws_bytes,
                            cc3_stream_t stream) {
  Plan p;
  int rc = common_checks(c, no, nv, nchol, prec, 0, ws, ws_bytes, &p);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1 for the Cholesky form");
  if (i < 0 || j < 0 || k < 0 || i >= no || j >= no || k >= no || (i == j && j == k))
    return fail(CC3_E_INVAL, "(%d,%d,%d) is not an ordered triple of distinct-enough indices < %d",
                i, j, k, no);
  const void* ptrs[] = {eps, L, t1, t2, tau};
  const char* names[] = {"eps", "L", "t1", "t2", "tau"};
  for (int a = 0; a < 5; ++a)
    if ((rc = check_dev_ptr(ptrs[a], names[a]))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws);
  std::lock_guard<std::mutex> g(c->mu);
  prepare_cholesky(c, p, w, L, t1, st);
  const int h[3] = {i, j, k};
  HIPCHK(hipMemcpyAsync(w.tri, h, sizeof h, hipMemcpyHostToDevice, st));
  launch_t2N(t2, w.t2N, no, nv, st);
  if (prec == CC3_FP64) {
    launch_wbuild(t2, w.t2N, w.b, w.tri, 1, w.cubes[0], no, nv, true, st);
  } else {
    launch_lp_convert(t2, w.b, no, nv, w.lp, st);
    launch_wbuild_lp(w.lp, w.tri, 1, w.cubes[0], no, nv, true, st);
  }
  launch_tau_export(eps, w.tri, w.cubes[0], tau, no, nv, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return CC3_OK;
}
