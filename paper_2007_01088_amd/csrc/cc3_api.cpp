// One-shot entry points of the C ABI (declared in include/cc3.h): argument
// checks, the workspace plan, and the launch sequence of one residual
// evaluation on the caller's stream (Algorithm 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <initializer_list>
#include <mutex>
#include <vector>

#include "cc3_host.hpp"

using namespace cc3;


extern "C" const char* cc3_last_error(void) { return last_error_str(); }

// ---------------------------------------------------------------------------
// The workspace of the allocation-free residual (cc3_triples_residual_noalloc):
// a static device array of this library, one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address, per device, comes from hipGetSymbolAddress at
// context creation and is the only form in which host code uses it.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES];

// With `device` current: look up this device's copy of the array once.
static int scratch_setup(int device) {
  if (device >= SCRATCH_MAX_DEVICES)
    return fail(CC3_E_INVAL, "device %d beyond the %d devices the scratch table holds", device,
                SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return CC3_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(CC3_E_DEVICE, "hipGetSymbolAddress of the scratch array failed on device %d: %s",
                device, hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return CC3_OK;
}

static void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return device >= 0 && device < SCRATCH_MAX_DEVICES ? g_scratch_ptr[device] : nullptr;
}

extern "C" int cc3_create(cc3_ctx** out, int device) {
  if (!out) return fail(CC3_E_INVAL, "cc3_create: out is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n)
    return fail(CC3_E_INVAL, "cc3_create: device %d out of range (%d devices)", device, n);
  {
    int prev = 0;
    HIPCHK(hipGetDevice(&prev));
    HIPCHK(hipSetDevice(device));
    const int rc = scratch_setup(device);
    (void)hipSetDevice(prev);
    if (rc) return rc;
  }
  cc3_ctx* c = new cc3_ctx();
  c->device = device;
  *out = c;
  return CC3_OK;
}

extern "C" int cc3_destroy(cc3_ctx* c) {
  if (!c) return CC3_OK;
  c->prof.destroy();
  c->run.destroy();
  delete c;
  return CC3_OK;
}

extern "C" int cc3_profile_enable(cc3_ctx* c, int on) {
  if (!c) return fail(CC3_E_INVAL, "cc3_profile_enable: ctx is NULL");
  std::lock_guard<std::mutex> g(c->mu);
  c->prof.reset();
  c->prof.on = on != 0;
  return CC3_OK;
}

extern "C" int cc3_profile_get(cc3_ctx* c, cc3_kernel_stat* out, int max, int* count) {
  if (!c || !out || !count || max < 0) return fail(CC3_E_INVAL, "cc3_profile_get: bad argument");
  std::lock_guard<std::mutex> g(c->mu);
  return c->prof.collect(out, max, count);
}

extern "C" int cc3_workspace_size(int no, int nv, int nchol, int prec, unsigned flags,
                                  size_t* bytes) {
  if (!bytes) return fail(CC3_E_INVAL, "cc3_workspace_size: bytes is NULL");
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  Plan p;
  make_plan_ex(no, nv, nchol, prec, flags, true, 0, &p);
  *bytes = p.total;
  return CC3_OK;
}

extern "C" int cc3_batch_plan(int no, int nv, int nchol, int prec, unsigned flags,
                              int* triples_per_batch, int* nbatches) {
  if (!triples_per_batch || !nbatches) return fail(CC3_E_INVAL, "cc3_batch_plan: NULL output");
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  Plan p;
  make_plan_ex(no, nv, nchol, prec, flags, true, 0, &p);
  *triples_per_batch = p.batch;
  *nbatches = (p.ntri + p.batch - 1) / p.batch;
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

extern "C" int cc3_cvs_triples(int no, const int32_t* core, int ncore, int32_t* triples,
                               int capacity, int* ntriples) {
  if (no < 1 || no > 63) return fail(CC3_E_INVAL, "cc3_cvs_triples: no must be in [1, 63] (got %d)", no);
  if (ncore < 0 || (ncore > 0 && !core)) return fail(CC3_E_INVAL, "cc3_cvs_triples: bad core list");
  if (!ntriples) return fail(CC3_E_INVAL, "cc3_cvs_triples: ntriples is NULL");
  bool is_core[64] = {};
  for (int c = 0; c < ncore; ++c) {
    if (core[c] < 0 || core[c] >= no)
      return fail(CC3_E_INVAL, "cc3_cvs_triples: core index %d outside [0, %d)", core[c], no);
    is_core[core[c]] = true;
  }
  int n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      *ntriples = n;
      if (!triples) return CC3_OK;
      if (capacity < n)
        return fail(CC3_E_INVAL, "cc3_cvs_triples: capacity %d below the count %d", capacity, n);
      n = 0;
    }
    for (int i = 0; i < no; ++i)
      for (int j = 0; j <= i; ++j)
        for (int k = 0; k <= j; ++k) {
          if ((i == j && j == k) || !(is_core[i] || is_core[j] || is_core[k])) continue;
          if (pass == 1) {
            triples[3 * n] = i;
            triples[3 * n + 1] = j;
            triples[3 * n + 2] = k;
          }
          ++n;
        }
  }
  return CC3_OK;
}

// Host-memory arguments of the one-shot calls.  An input in host memory is
// copied on the call's stream into a workspace staging area, and the kernels read
// the copy; an output in host memory is produced in a staging area and copied
// back, and the call then waits for its stream, so that the caller's host
// buffers hold the results (and may be reused) when it returns.
struct HostArgs {
  struct Out {
    double* dev;   // where the kernels write
    double* host;  // the caller's host buffer, or null for device memory
    size_t n;
  };
  hipStream_t st;
  bool any = false;
  // On return `p` points at device memory holding the input.
  int in(const double*& p, const char* what, double* stage, size_t n) {
    bool host = false;
    int rc = classify_ptr(p, what, &host);
    if (rc || !host) return rc;
    HIPCHK(hipMemcpyAsync(stage, p, n * sizeof(double), hipMemcpyHostToDevice, st));
    p = stage;
    any = true;
    return CC3_OK;
  }
  int out(double* p, const char* what, double* stage, size_t n, Out& o) {
    bool host = false;
    int rc = classify_ptr(p, what, &host);
    if (rc) return rc;
    o.n = n;
    o.host = host ? p : nullptr;
    o.dev = host ? stage : p;
    any = any || host;
    return CC3_OK;
  }
  // the caller's current values, for CC3_ACCUMULATE into a host output
  int preload(const Out& o) {
    if (o.host) HIPCHK(hipMemcpyAsync(o.dev, o.host, o.n * sizeof(double), hipMemcpyHostToDevice, st));
    return CC3_OK;
  }
  int finish(std::initializer_list<const Out*> outs) {
    for (const Out* o : outs)
      if (o->host)
        HIPCHK(hipMemcpyAsync(o->host, o->dev, o->n * sizeof(double), hipMemcpyDeviceToHost, st));
    if (any) HIPCHK(hipStreamSynchronize(st));
    return CC3_OK;
  }
};

// Staging area of a host L: the cube region after the Cholesky scratch.
static double* stage_L(const Plan& p, void* ws) {
  return (double*)((char*)ws + p.off_cubes + p.chol_bytes);
}

// eps, L (Cholesky form only), t1 and t2 onto the device.
static int stage_inputs(HostArgs& h, const Plan& p, const Ws& w, void* ws, const double*& eps,
                        const double*& L, const double*& t1, const double*& t2) {
  const size_t o = p.no, v = p.nv, J = p.nchol;
  int rc;
  if ((rc = h.in(eps, "eps", w.st_eps, o + v))) return rc;
  if (J && (rc = h.in(L, "L", stage_L(p, ws), J * (o + v) * (o + v)))) return rc;
  if (t1 && (rc = h.in(t1, "t1", w.st_t1, o * v))) return rc;
  return h.in(t2, "t2", w.st_t2, o * o * v * v);
}

// The integral blocks of a blocks-form call (paper index order, device or host)
// into the internal layouts of the workspace.  Host blocks pass through the cube
// region: the small ones whole, then slabs of the first virtual index of g_vvvo
// and g_vvov (as many as fit).
static int load_blocks(Profiler* pf, HostArgs& h, const Plan& p, const Ws& w, void* ws,
                       const double* g_vvvo, const double* g_oovo, const double* g_ovov,
                       const double* g_ooov, const double* g_vvov, const double* F_ov,
                       hipStream_t st) {
  const int no = p.no, nv = p.nv;
  const size_t o = no, v = nv;
  int rc;
  {
    Timer tm(pf, st, FAM_BUILD, 0.0, 0.0);
    // host blocks pass through the cube region: the small ones whole, then
    // slabs of the first virtual index of g_vvvo and g_vvov
    char* cr = (char*)ws + p.off_cubes;
    const size_t b3 = (o * o * o * v * 8 + 255) & ~(size_t)255;
    const size_t b2 = (o * o * v * v * 8 + 255) & ~(size_t)255;
    const size_t b1 = (o * v * 8 + 255) & ~(size_t)255;
    if ((rc = h.in(g_oovo, "g_oovo", (double*)cr, o * o * o * v))) return rc;
    if ((rc = h.in(g_ooov, "g_ooov", (double*)(cr + b3), o * o * o * v))) return rc;
    if ((rc = h.in(g_ovov, "g_ovov", (double*)(cr + 2 * b3), o * o * v * v))) return rc;
    if ((rc = h.in(F_ov, "F_ov", (double*)(cr + 2 * b3 + b2), o * v))) return rc;
    launch_relayout_small(g_oovo, g_ovov, g_ooov, F_ov, w.b, no, nv, st);
    bool hv = false, hw = false;
    if ((rc = classify_ptr(g_vvvo, "g_vvvo", &hv)) || (rc = classify_ptr(g_vvov, "g_vvov", &hw)))
      return rc;
    const size_t slab = o * v * v;  // doubles per first index of g_vvvo and g_vvov
    int ny = nv;
    if (hv || hw) {
      const size_t small = 2 * b3 + b2 + b1, region = p.total - p.off_cubes;
      const size_t fit = (region - small) / (2 * ((slab * 8 + 255) & ~(size_t)255));
      ny = (int)std::max<size_t>(1, std::min<size_t>(nv, fit));
      const char* cap = getenv("CC3_STAGE_Y");  // smaller slabs (tests of the staging)
      if (cap && atoi(cap) > 0) ny = std::min(ny, atoi(cap));
    }
    double* sa = (double*)(cr + 2 * b3 + b2 + b1);
    double* sb = sa + (size_t)ny * slab;
    for (int y0 = 0; y0 < nv; y0 += ny) {
      const int n = std::min(ny, nv - y0);
      const double* a = g_vvvo + (size_t)y0 * slab;
      const double* b = g_vvov + (size_t)y0 * slab;
      if (hv) {
        HIPCHK(hipMemcpyAsync(sa, a, n * slab * 8, hipMemcpyHostToDevice, st));
        a = sa;
      }
      if (hw) {
        HIPCHK(hipMemcpyAsync(sb, b, n * slab * 8, hipMemcpyHostToDevice, st));
        b = sb;
      }
      launch_relayout_vv(a, b, y0, n, w.b, no, nv, st);
    }
    h.any = h.any || hv || hw;
    launch_gcb(w.b, no, nv, st);
  }
  return CC3_OK;
}

static int common_checks(cc3_ctx* c, int no, int nv, int nchol, int prec, unsigned flags,
                         void* ws, size_t ws_bytes, Plan* p) {
  if (!c) return fail(CC3_E_INVAL, "ctx is NULL");
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  if (flags & ~(unsigned)(CC3_ACCUMULATE | CC3_CHECK | CC3_ONE_STREAM | CC3_LOWP_CONTRACT |
                         CC3_DETERMINISTIC))
    return fail(CC3_E_INVAL, "unknown flag bits 0x%x", flags);
  if ((flags & CC3_LOWP_CONTRACT) && prec == CC3_FP64)
    return fail(CC3_E_INVAL, "CC3_LOWP_CONTRACT needs a low precision (FP32, BF16X3, BF16X6)");
  make_plan_ex(no, nv, nchol, prec, flags, true, 0, p);
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
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  const size_t o = no, v = nv;
  const bool acc = (flags & CC3_ACCUMULATE) != 0;
  std::lock_guard<std::mutex> g(c->mu);
  HostArgs h{st};
  HostArgs::Out O1, O2;
  if ((rc = stage_inputs(h, p, w, ws, eps, L, t1, t2))) return rc;
  if ((rc = h.out(omega1, "omega1", w.st_o1, o * v, O1))) return rc;
  if ((rc = h.out(omega2, "omega2", w.t2N, o * o * v * v, O2))) return rc;  // t2N is free by then
  if (acc && (rc = h.preload(O1))) return rc;
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
  if ((rc = residual_from_blocks(c->run, &c->prof, p, w, eps, t2, O1.dev, O2.dev, acc, st,
                                 acc ? O2.host : nullptr)))
    return rc;
  return h.finish({&O1, &O2});
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
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  const size_t o = no, v = nv;
  const bool acc = (flags & CC3_ACCUMULATE) != 0;
  std::lock_guard<std::mutex> g(c->mu);
  HostArgs h{st};
  HostArgs::Out O1, O2;
  const double* none = nullptr;
  if ((rc = stage_inputs(h, p, w, ws, eps, none, none, t2))) return rc;
  if ((rc = h.out(omega1, "omega1", w.st_o1, o * v, O1))) return rc;
  if ((rc = h.out(omega2, "omega2", w.t2N, o * o * v * v, O2))) return rc;
  if (acc && (rc = h.preload(O1))) return rc;
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, nullptr, t2, st))) return rc;
  if ((rc = load_blocks(&c->prof, h, p, w, ws, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, st)))
    return rc;
  if ((rc = residual_from_blocks(c->run, &c->prof, p, w, eps, t2, O1.dev, O2.dev, acc, st,
                                 acc ? O2.host : nullptr)))
    return rc;
  return h.finish({&O1, &O2});
}

// Unordered triples i >= j >= k, not all equal, below no.
static int check_triples(const Plan& p, const int32_t* triples, int ntriples) {
  if (ntriples < 0 || ntriples > p.ntri)
    return fail(CC3_E_INVAL, "ntriples %d out of range [0, %d]", ntriples, p.ntri);
  if (ntriples > 0 && !triples) return fail(CC3_E_INVAL, "triples is NULL");
  for (int t = 0; t < ntriples; ++t) {
    const int i = triples[3 * t], j = triples[3 * t + 1], k = triples[3 * t + 2];
    if (!(i < p.no && i >= j && j >= k && k >= 0) || (i == j && j == k))
      return fail(CC3_E_INVAL, "triple %d = (%d,%d,%d) is not an unordered triple i>=j>=k "
                  "(not all equal) below no=%d", t, i, j, k, p.no);
  }
  return CC3_OK;
}

// The contravariant residual of the listed triples, once the integral blocks are in
// place: Ot <- 0, the batched loop over the list, Ot~2 = Ot2 + OtT^T, outputs.
static int subset_from_blocks(cc3_ctx* c, const Plan& p, const Ws& w, HostArgs& h,
                              const double* eps, const double* t2, const int32_t* triples,
                              int ntriples, HostArgs::Out& O1, HostArgs::Out& O2, hipStream_t st) {
  const int no = p.no, nv = p.nv;
  int rc;
  launch_fill(w.Ot1, (int64_t)no * nv, 0.0, st);
  launch_fill(w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
  launch_fill(w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
  if (ntriples > 0) {
    HIPCHK(hipMemcpyAsync(w.tri, triples, sizeof(int) * 3 * (size_t)ntriples,
                          hipMemcpyHostToDevice, st));
    if ((rc = triple_loop(c->run, &c->prof, p, w, eps, t2, w.tri, triples, ntriples, st)))
      return rc;
  }
  launch_combine(w.Ot1, w.Ot2, w.OtT, O1.dev, O2.dev, no, nv, st);
  HIPCHK(hipGetLastError());
  if ((rc = h.finish({&O1, &O2}))) return rc;
  HIPCHK(hipStreamSynchronize(st));  // the host triples were copied on st
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
  if ((rc = check_triples(p, triples, ntriples))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  HostArgs h{st};
  HostArgs::Out O1, O2;
  if ((rc = stage_inputs(h, p, w, ws, eps, L, t1, t2))) return rc;
  if ((rc = h.out(omega1_tilde, "omega1_tilde", w.st_o1, (size_t)no * nv, O1))) return rc;
  if ((rc = h.out(omega2_tilde, "omega2_tilde", w.t2N, (size_t)no * no * nv * nv, O2))) return rc;
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
  return subset_from_blocks(c, p, w, h, eps, t2, triples, ntriples, O1, O2, st);
}

extern "C" int cc3_triples_residual_subset_blocks(
    cc3_ctx* c, int no, int nv, const double* eps, const double* g_vvvo, const double* g_oovo,
    const double* g_ovov, const double* g_ooov, const double* g_vvov, const double* F_ov,
    const double* t2, const int32_t* triples, int ntriples, double* omega1_tilde,
    double* omega2_tilde, int prec, unsigned flags, void* ws, size_t ws_bytes,
    cc3_stream_t stream) {
  Plan p;
  int rc = common_checks(c, no, nv, 0, prec, flags, ws, ws_bytes, &p);
  if (rc) return rc;
  if ((rc = check_triples(p, triples, ntriples))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  HostArgs h{st};
  HostArgs::Out O1, O2;
  const double* none = nullptr;
  if ((rc = stage_inputs(h, p, w, ws, eps, none, none, t2))) return rc;
  if ((rc = h.out(omega1_tilde, "omega1_tilde", w.st_o1, (size_t)no * nv, O1))) return rc;
  if ((rc = h.out(omega2_tilde, "omega2_tilde", w.t2N, (size_t)no * no * nv * nv, O2))) return rc;
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, nullptr, t2, st))) return rc;
  if ((rc = load_blocks(&c->prof, h, p, w, ws, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, st)))
    return rc;
  return subset_from_blocks(c, p, w, h, eps, t2, triples, ntriples, O1, O2, st);
}

// tau^{abc}_{ijk} of one ordered triple once the integral blocks are in place.
static int t3_from_blocks(const Plan& p, const Ws& w, HostArgs& hs, const double* eps,
                          const double* t2, int i, int j, int k, HostArgs::Out& T,
                          hipStream_t st) {
  const int no = p.no, nv = p.nv;
  int rc;
  const int h[3] = {i, j, k};
  HIPCHK(hipMemcpyAsync(w.tri, h, sizeof h, hipMemcpyHostToDevice, st));
  launch_t2N(t2, w.t2N, no, nv, st);
  if (p.prec == CC3_FP64) {
    launch_wbuild(t2, w.t2N, w.b, w.tri, 1, w.cubes[0], no, nv, true, st);
  } else {
    launch_lp_convert(t2, w.b, no, nv, w.lp, st);
    launch_wbuild_lp(w.lp, w.tri, 1, w.cubes[0], no, nv, true, st);
  }
  launch_tau_export(eps, w.tri, w.cubes[0], T.dev, no, nv, st);
  HIPCHK(hipGetLastError());
  if ((rc = hs.finish({&T}))) return rc;
  HIPCHK(hipStreamSynchronize(st));  // the host triple was copied on st
  return CC3_OK;
}

static int check_ordered(int no, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= no || j >= no || k >= no || (i == j && j == k))
    return fail(CC3_E_INVAL, "(%d,%d,%d) is not an ordered triple of indices < %d, not all equal",
                i, j, k, no);
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
  if ((rc = check_ordered(no, i, j, k))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  HostArgs hs{st};
  HostArgs::Out T;
  if ((rc = stage_inputs(hs, p, w, ws, eps, L, t1, t2))) return rc;
  // a host tau is produced in the second cube buffer set, unused by this call
  if ((rc = hs.out(tau, "tau", w.cubes[1], (size_t)nv * nv * nv, T))) return rc;
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
  return t3_from_blocks(p, w, hs, eps, t2, i, j, k, T, st);
}

extern "C" int cc3_t3_block_blocks(cc3_ctx* c, int no, int nv, const double* eps,
                                   const double* g_vvvo, const double* g_oovo,
                                   const double* g_ovov, const double* g_ooov,
                                   const double* g_vvov, const double* F_ov, const double* t2,
                                   int i, int j, int k, double* tau, int prec, void* ws,
                                   size_t ws_bytes, cc3_stream_t stream) {
  Plan p;
  int rc = common_checks(c, no, nv, 0, prec, 0, ws, ws_bytes, &p);
  if (rc) return rc;
  if ((rc = check_ordered(no, i, j, k))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  HostArgs hs{st};
  HostArgs::Out T;
  const double* none = nullptr;
  if ((rc = stage_inputs(hs, p, w, ws, eps, none, none, t2))) return rc;
  // a host tau is produced in the second cube buffer set; host blocks staged through the
  // cube region have been consumed (earlier on the same stream) when the export writes it
  if ((rc = hs.out(tau, "tau", w.cubes[1], (size_t)nv * nv * nv, T))) return rc;
  if ((rc = load_blocks(&c->prof, hs, p, w, ws, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, st)))
    return rc;
  return t3_from_blocks(p, w, hs, eps, t2, i, j, k, T, st);
}

extern "C" int cc3_jacobian_prep(cc3_ctx* c, int no, int nv, int nchol, const double* eps,
                                 const double* L, const double* t1, const double* t2, double* zv,
                                 double* zo, int prec, unsigned flags, void* ws, size_t ws_bytes,
                                 cc3_stream_t stream) {
  if (flags & CC3_LOWP_CONTRACT)
    return fail(CC3_E_INVAL, "CC3_LOWP_CONTRACT applies to the residual calls only");
  Plan p;
  int rc = common_checks(c, no, nv, nchol, prec, flags, ws, ws_bytes, &p);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1 for the Cholesky form");
  if ((int64_t)no * no * nv * nv >= ((int64_t)1 << 31))
    return fail(CC3_E_INVAL, "no^2 nv^2 must stay below 2^31 for the Jacobian preparation "
                "(no=%d nv=%d)", no, nv);
  const void* ptrs[] = {eps, L, t1, t2, zv, zo};
  const char* names[] = {"eps", "L", "t1", "t2", "zv", "zo"};
  for (int i = 0; i < 6; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
  return jacobian_prep_from_blocks(c->run, &c->prof, p, w, eps, t2, zv, zo,
                                   (flags & CC3_ACCUMULATE) != 0, st);
}

// ---------------------------------------------------------------------------
// Allocation-free residual
// ---------------------------------------------------------------------------
extern "C" int cc3_triples_residual_noalloc(cc3_ctx* c, int no, int nv, int nchol,
                                            const double* eps, const double* L, const double* t1,
                                            const double* t2, double* omega1, double* omega2,
                                            int prec, unsigned flags, cc3_stream_t stream) {
  if (!c) return fail(CC3_E_INVAL, "ctx is NULL");
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1 for the Cholesky form");
  if (flags & ~(unsigned)(CC3_ACCUMULATE | CC3_ONE_STREAM | CC3_LOWP_CONTRACT | CC3_DETERMINISTIC))
    return fail(CC3_E_INVAL, "flags 0x%x: the allocation-free call accepts CC3_ACCUMULATE, "
                "CC3_ONE_STREAM, CC3_LOWP_CONTRACT and CC3_DETERMINISTIC", flags);
  if ((flags & CC3_LOWP_CONTRACT) && prec == CC3_FP64)
    return fail(CC3_E_INVAL, "CC3_LOWP_CONTRACT needs a low precision (FP32, BF16X3, BF16X6)");
  HIPCHK(hipSetDevice(c->device));
  const void* ptrs[] = {eps, L, t1, t2, omega1, omega2};
  const char* names[] = {"eps", "L", "t1", "t2", "omega1", "omega2"};
  for (int i = 0; i < 6; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  void* ws = scratch_ptr(c->device);
  if (!ws) return fail(CC3_E_DEVICE, "the scratch array of device %d was not set up", c->device);
  // the plan of the one-shot call, with fewer triples per batch until it fits the array
  Plan p;
  make_plan_ex(no, nv, nchol, prec, flags, true, 0, &p);
  const size_t per_triple = 5 * p.cube * sizeof(double);
  for (int b = p.batch - 1; p.total > SCRATCH_BYTES && b >= 1; --b)
    make_plan_ex(no, nv, nchol, prec, flags, true, (size_t)b * per_triple, &p);
  if (p.total > SCRATCH_BYTES)
    return fail(CC3_E_NOMEM, "no=%d nv=%d nchol=%d needs %zu bytes of workspace at one triple per "
                "batch; the allocation-free call has %zu", no, nv, nchol, p.total, SCRATCH_BYTES);
  p.flags |= PLAN_CALLER_STREAM;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  if ((rc = prepare_cholesky(nullptr, p, w, L, t1, st))) return rc;
  return residual_from_blocks(c->run, nullptr, p, w, eps, t2, omega1, omega2,
                              (flags & CC3_ACCUMULATE) != 0, st);
}
