// One-shot entry points of the C ABI (declared in include/cc3.h): argument
// checks, the workspace plan, and the launch sequence of one residual
// evaluation on the caller's stream (Algorithm 1).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "cc3_host.hpp"

using namespace cc3;

struct cc3_ctx {
  int device;
  Profiler prof;
  Runner run;
  std::mutex mu;
};

extern "C" const char* cc3_last_error(void) { return last_error_str(); }

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
  const void* ptrs[] = {eps, L, t1, t2, omega1, omega2};
  const char* names[] = {"eps", "L", "t1", "t2", "omega1", "omega2"};
  for (int i = 0; i < 6; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
  return residual_from_blocks(c->run, &c->prof, p, w, eps, t2, omega1, omega2,
                              (flags & CC3_ACCUMULATE) != 0, st);
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
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, nullptr, t2, st))) return rc;
  {
    Timer tm(&c->prof, st, FAM_BUILD, 0.0, 0.0);
    launch_relayout_blocks(g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, w.b, no, nv, st);
  }
  return residual_from_blocks(c->run, &c->prof, p, w, eps, t2, omega1, omega2,
                              (flags & CC3_ACCUMULATE) != 0, st);
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
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  if ((flags & CC3_CHECK) && (rc = run_input_check(p, w, eps, L, t2, st))) return rc;
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
  launch_fill(w.Ot1, (int64_t)no * nv, 0.0, st);
  launch_fill(w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
  launch_fill(w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
  if (ntriples > 0) {
    HIPCHK(hipMemcpyAsync(w.tri, triples, sizeof(int) * 3 * (size_t)ntriples,
                          hipMemcpyHostToDevice, st));
    if ((rc = triple_loop(c->run, &c->prof, p, w, eps, t2, w.tri, triples, ntriples, st)))
      return rc;
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
  Ws w = carve(p, ws, nullptr);
  std::lock_guard<std::mutex> g(c->mu);
  if ((rc = prepare_cholesky(&c->prof, p, w, L, t1, st))) return rc;
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
