// Host-side core of libcc3: error reporting, kernel timing, the two-stream
// runner, the workspace plan and the launch sequence of one residual
// evaluation of Algorithm 1 (T1 transformation and integral blocks, the
// batched restricted triple loop, the covariant back-transformation).
#include "cc3_host.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace cc3 {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error_str() { return g_err.c_str(); }

int check_sizes(int no, int nv, int nchol, int prec) {
  if (no < 1 || nv < 1) return fail(CC3_E_INVAL, "sizes must be positive (no=%d nv=%d)", no, nv);
  if (nchol < 0) return fail(CC3_E_INVAL, "nchol must be >= 0 (got %d)", nchol);
  if (no > 63 || nv > 1024)
    return fail(CC3_E_INVAL, "sizes beyond the supported range no <= 63, nv <= 1024 (no=%d nv=%d)",
                no, nv);
  if (prec != CC3_FP64 && prec != CC3_FP32 && prec != CC3_BF16X3 && prec != CC3_BF16X6)
    return fail(CC3_E_INVAL, "unknown precision %d", prec);
  return CC3_OK;
}

int check_dev_ptr(const void* p, const char* what) {
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

int classify_ptr(const void* p, const char* what, bool* host) {
  if (!p) return fail(CC3_E_INVAL, "%s is NULL", what);
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // unregistered (pageable) host memory
    *host = true;
    return CC3_OK;
  }
  *host = !(a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged);
  return CC3_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
const char* kFamilies[NFAM] = {"t1_transform", "block_build",    "w_build",       "mix",
                               "omega_contract", "reduce",        "back_transform", "jacobian_prep",
                               "omega_oo",       "l3_build",      "density_contract"};

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::reset() {
  for (auto& t : timed) { pool.push_back(t.start); pool.push_back(t.stop); }
  timed.clear();
}

int Profiler::collect(cc3_kernel_stat* out, int max, int* count) {
  cc3_kernel_stat st[NFAM];
  memset(st, 0, sizeof st);
  for (int f = 0; f < NFAM; ++f) snprintf(st[f].name, sizeof st[f].name, "%s", kFamilies[f]);
  for (auto& t : timed) {
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

void Profiler::destroy() {
  for (auto& t : timed) { hipEventDestroy(t.start); hipEventDestroy(t.stop); }
  for (auto e : pool) hipEventDestroy(e);
  timed.clear();
  pool.clear();
}

Timer::Timer(Profiler* pf_, hipStream_t st_, int fam, double flops, double bytes)
    : pf(pf_), st(st_) {
  on = pf && pf->on;
  if (!on) return;
  tl.family = fam;
  tl.flops = flops;
  tl.bytes = bytes;
  tl.start = pf->take();
  tl.stop = pf->take();
  if (!tl.start || !tl.stop) { on = false; return; }
  hipEventRecord(tl.start, st);
}

Timer::~Timer() {
  if (!on) return;
  hipEventRecord(tl.stop, st);
  pf->timed.push_back(tl);
}

// ---------------------------------------------------------------------------
// runner
// ---------------------------------------------------------------------------
int Runner::init(hipStream_t s0) {
  if (ready) return CC3_OK;
  own0 = (s0 == nullptr);
  if (!own0) s[0] = s0;
  for (int k = 0; k < NSTREAM; ++k) {
    if ((k > 0 || own0) && hipStreamCreateWithFlags(&s[k], hipStreamNonBlocking) != hipSuccess)
      return fail(CC3_E_DEVICE, "could not create the internal streams");
    if (hipEventCreateWithFlags(&ev_done[k], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_red[k], hipEventDisableTiming) != hipSuccess)
      return fail(CC3_E_DEVICE, "could not create the internal streams");
  }
  if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess)
    return fail(CC3_E_DEVICE, "could not create the internal streams");
  ready = true;
  return CC3_OK;
}

void Runner::destroy() {
  if (!ready) return;
  for (int k = 0; k < NSTREAM; ++k) {
    if (k > 0 || own0) hipStreamDestroy(s[k]);
    hipEventDestroy(ev_done[k]);
    hipEventDestroy(ev_red[k]);
  }
  hipEventDestroy(ev_fork);
  ready = false;
}

// ---------------------------------------------------------------------------
// plan and workspace
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int env_int(const char* name, int dflt) {
  const char* s = getenv(name);
  if (!s || !*s) return dflt;
  int v = atoi(s);
  return v > 0 ? v : dflt;
}

size_t block_bytes(int no, int nv) {
  const size_t o = no, v = nv;
  return align256(o * v * v * v * 8) + align256(o * (v + o) * v * v * 8) * 2 +
         align256(o * o * o * v * 8) * 2 + align256(o * o * v * v * 8) + align256(o * v * 8);
}

Blocks carve_blocks(int no, int nv, void* base) {
  const size_t o = no, v = nv;
  char* b = (char*)base;
  Blocks bl;
  bl.Gw = (double*)b; b += align256(o * v * v * v * 8);
  bl.Gbc = (double*)b; b += align256(o * (v + o) * v * v * 8);
  bl.Gcb = (double*)b; b += align256(o * (v + o) * v * v * 8);
  bl.Go = (double*)b; b += align256(o * o * o * v * 8);
  bl.Hs = (double*)b; b += align256(o * o * o * v * 8);
  bl.Jo = (double*)b; b += align256(o * o * v * v * 8);
  bl.F = (double*)b;
  return bl;
}

int make_plan_ex(int no, int nv, int nchol, int prec, unsigned flags, bool with_blocks,
                 size_t cube_budget, Plan* p) {
  memset(p, 0, sizeof *p);
  p->no = no; p->nv = nv; p->nchol = nchol; p->prec = prec; p->flags = flags;
  const size_t o = no, v = nv, J = nchol;
  p->ntri = (int)((size_t)no * (no + 1) * (no + 2) / 6 - no);
  p->cube = (size_t)cube_slot(nv);  // one padded cube slot
  // triples per batch: enough W-build workgroups per launch to fill 256 CUs
  // many times over, and at least min(no, 16) triples, so that the kernels that
  // are parallel over the first occupied index p (the oo contraction, the
  // reductions) find pairs for many p in every batch; bounded by a cube-memory
  // budget per buffer set (32 GiB by default: 12 triples at nv = 400)
  const size_t wg_per_triple = 3 * v * ((v + 127) / 128) * ((v + 127) / 128);
  int batch = (int)std::max<size_t>(1, (size_t)(12288 + wg_per_triple - 1) / wg_per_triple);
  batch = std::max(batch, std::min(no, 8));
  const size_t budget =
      cube_budget ? cube_budget : ((size_t)env_int("CC3_CUBE_BUDGET_MB", 32768) << 20);
  const size_t per_triple = 5 * p->cube * sizeof(double);
  batch = (int)std::min<size_t>((size_t)batch, std::max<size_t>(1, budget / per_triple));
  batch = env_int("CC3_BATCH", batch);
  batch = std::min(batch, MAX_BATCH);  // bounds the kernels' per-p pair lists
  batch = std::max(1, std::min(batch, std::max(1, p->ntri)));
  // balanced: the loop is split into ceil(ntri / batch) batches whose sizes differ by at
  // most one, and `batch` becomes the largest of them
  if (p->ntri > 0) {
    const int nb = (p->ntri + batch - 1) / batch;
    batch = (p->ntri + nb - 1) / nb;
  }
  p->batch = batch;
  // largest (triples x chunks) product over the batch sizes the loop can see
  size_t tc = 1;
  for (int nb = 1; nb <= batch; ++nb)
    tc = std::max(tc, (size_t)nb * std::max(omega_kchunks(nv, nb, (flags & CC3_LOWP_CONTRACT) != 0),
                                            zo_nbchunks(nv, nb)));
  p->pvv_entries = tc;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = align256(off + bytes); return at; };
  p->off_blocks = with_blocks ? take(block_bytes(no, nv)) : 0;
  p->off_Ot1 = take(o * v * 8);
  p->off_Ot2 = take(o * o * v * v * 8);
  p->off_OtT = take(o * o * v * v * 8);
  p->off_t2N = take(o * o * v * v * 8);
  p->off_lp = take(lp_operand_bytes(prec, no, nv));
  // partial slabs: Omega chunks of nv x (nv + 1), or Jacobian-preparation chunks of nv x no
  p->pvv_bytes = align256(tc * 6 * v * std::max(v + 1, o) * 8);
  p->off_Pvv = take(2 * p->pvv_bytes);
  if (flags & CC3_LOWP_CONTRACT) {
    if (prec == CC3_FP32) {
      p->gf_bytes = align256(o * (v + o) * v * v * 4);
      p->cubef_bytes = align256((size_t)batch * 2 * p->cube * 4);
    } else {
      p->gf_bytes = align256(lp_contract_g_bytes(prec, no, nv));
      p->cubef_bytes = align256((size_t)batch * lp_contract_cube_bytes(prec, nv));
    }
    p->off_gf = take(2 * p->gf_bytes);
    p->off_cubef = take(2 * p->cubef_bytes);
  }
  p->off_tri = take((size_t)std::max(1, p->ntri) * 3 * sizeof(int) + 64);
  p->off_flag = take(64);
  // the Cholesky scratch is dead once the blocks are built: it shares the cube region
  p->chol_bytes = J ? align256(J * v * v * 8) + align256(J * o * o * 8) * 2 +
                          align256(J * o * v * 8) * 2 + align256(J * 8) + align256(J * o * o * 8)
                    : 0;
  p->cube_bytes = align256((size_t)batch * 5 * p->cube * 8);
  size_t region = std::max(p->chol_bytes, 2 * p->cube_bytes);
  if (with_blocks) {
    const size_t nmo = o + v;
    p->off_stage = take(align256(nmo * 8) + 2 * align256(o * v * 8) + align256(o * o * v * v * 8));
    // setup-time staging in the cube region: a host L after the Cholesky scratch,
    // or the small host blocks plus one y slab of g_vvvo and of g_vvov
    const size_t small = 2 * align256(o * o * o * v * 8) + align256(o * o * v * v * 8) +
                         align256(o * v * 8);
    p->stage_region = std::max(p->chol_bytes + align256(J * nmo * nmo * 8),
                               small + 2 * align256(o * v * v * 8));
    region = std::max(region, p->stage_region);
  }
  p->off_cubes = take(region);
  p->off_chol = p->off_cubes;
  p->total = off;
  return CC3_OK;
}

Ws carve(const Plan& p, void* ws, const Blocks* external_blocks) {
  char* base = (char*)ws;
  Ws w;
  w.b = external_blocks ? *external_blocks : carve_blocks(p.no, p.nv, base + p.off_blocks);
  w.Ot1 = (double*)(base + p.off_Ot1);
  w.Ot2 = (double*)(base + p.off_Ot2);
  w.OtT = (double*)(base + p.off_OtT);
  w.t2N = (double*)(base + p.off_t2N);
  lp_operand_ptrs(p.prec, p.no, p.nv, base + p.off_lp, w.lp);
  for (int k = 0; k < 2; ++k) {
    w.Pvv[k] = (double*)(base + p.off_Pvv + k * p.pvv_bytes);
    w.cubes[k] = (double*)(base + p.off_cubes + k * p.cube_bytes);
  }
  w.GbcX = w.GcbX = w.cubesX[0] = w.cubesX[1] = nullptr;
  if (p.gf_bytes) {
    w.GbcX = base + p.off_gf;
    w.GcbX = base + p.off_gf + p.gf_bytes;
    for (int k = 0; k < 2; ++k) w.cubesX[k] = base + p.off_cubef + k * p.cubef_bytes;
  }
  w.tri = (int*)(base + p.off_tri);
  w.flag = (int*)(base + p.off_flag);
  w.st_eps = w.st_t1 = w.st_t2 = w.st_o1 = nullptr;
  if (p.stage_region) {
    const size_t o = p.no, v = p.nv;
    char* s = base + p.off_stage;
    w.st_eps = (double*)s; s += align256((o + v) * 8);
    w.st_t1 = (double*)s; s += align256(o * v * 8);
    w.st_o1 = (double*)s; s += align256(o * v * 8);
    w.st_t2 = (double*)s;
  }
  const size_t J = p.nchol, o = p.no, v = p.nv;
  char* c = base + p.off_chol;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* at = c + off; off = align256(off + bytes); return (double*)at; };
  w.cs.Lvv = take(J * v * v * 8);
  w.cs.Loo = take(J * o * o * 8);
  w.cs.LooT = take(J * o * o * 8);
  w.cs.LvoT = take(J * o * v * 8);
  w.cs.Lov = take(J * o * v * 8);
  w.cs.s = take(J * 8);
  w.cs.M = take(J * o * o * 8);
  return w;
}

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
static int nbatches(const Plan& p) { return (p.ntri + p.batch - 1) / p.batch; }

// Batch g of n triples split into nbatch batches whose sizes differ by at most one
// (the layout of the dealt triple table): first position and size.
static void batch_range(int n, int nbatch, int g, int* t0, int* nb) {
  const int q = n / nbatch, r = n % nbatch;
  *t0 = g * q + std::min(g, r);
  *nb = q + (g < r ? 1 : 0);
}

// Host copy of the device triple table (launch_triple_table): the restricted loop
// in lexicographic order, dealt round-robin over nbatch batches.
static void host_triples(int no, int nbatch, std::vector<int>& t) {
  std::vector<int> lex;
  for (int i = 0; i < no; ++i)
    for (int j = 0; j <= i; ++j)
      for (int k = 0; k <= j; ++k)
        if (!(i == j && j == k)) { lex.push_back(i); lex.push_back(j); lex.push_back(k); }
  const int n = (int)lex.size() / 3;
  nbatch = std::max(1, nbatch);
  t.assign(lex.size(), 0);
  for (int L = 0; L < n; ++L) {
    int t0, nb;
    batch_range(n, nbatch, L % nbatch, &t0, &nb);
    const int pos = t0 + L / nbatch;
    for (int c = 0; c < 3; ++c) t[3 * pos + c] = lex[3 * L + c];
  }
}

static int kind_of(int i, int j, int k) { return (i == j) ? 1 : (j == k) ? 2 : 0; }

int prepare_cholesky(Profiler* pf, const Plan& p, const Ws& w, const double* L, const double* t1,
                     hipStream_t st) {
  {
    Timer tm(pf, st, FAM_T1, 0.0, 0.0);
    launch_t1_transform(L, t1, w.cs, p.no, p.nv, p.nchol, st);
    launch_fock(t1, w.cs, w.b.F, p.no, p.nv, p.nchol, st);
  }
  {
    const double v = p.nv, o = p.no, J = p.nchol;
    const double fl = 2.0 * J * (2.0 * v * v * v * o + o * o * v * v + 2.0 * o * o * o * v);
    Timer tm(pf, st, FAM_BUILD, fl, 0.0);
    launch_build_blocks(w.cs, w.b, p.no, p.nv, p.nchol, st);
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

// The batched triple loop over a device triple table `tri` of n entries whose
// host copy is `ht` (for FLOP accounting only).  Batch b runs on runner
// stream b % 2 with buffer set b % 2; reduction b waits for reduction b - 1.
// Forks from and joins back to `st`.
// After a failure inside the batched loop: make `st` wait for whatever the runner
// streams hold (best effort, errors ignored), so that a caller that synchronises
// `st` before releasing the workspace also waits for work enqueued there.
static void join_runner(Runner& rn, hipStream_t st) {
  if (!rn.ready) return;
  for (int k = 0; k < NSTREAM; ++k) {
    if (hipEventRecord(rn.ev_done[k], rn.s[k]) == hipSuccess)
      (void)hipStreamWaitEvent(st, rn.ev_done[k], 0);
  }
  (void)hipGetLastError();
}

static int triple_loop_body(Runner& rn, Profiler* pf, const Plan& p, const Ws& w,
                            const double* eps, const double* t2, const int* tri, const int* ht,
                            int n, hipStream_t st);

int triple_loop(Runner& rn, Profiler* pf, const Plan& p, const Ws& w, const double* eps,
                const double* t2, const int* tri, const int* ht, int n, hipStream_t st) {
  if (p.flags & PLAN_CALLER_STREAM) return triple_loop_body(rn, pf, p, w, eps, t2, tri, ht, n, st);
  int rc = rn.init();
  if (rc) return rc;
  rc = triple_loop_body(rn, pf, p, w, eps, t2, tri, ht, n, st);
  if (rc) join_runner(rn, st);
  return rc;
}

static int triple_loop_body(Runner& rn, Profiler* pf, const Plan& p, const Ws& w,
                            const double* eps, const double* t2, const int* tri, const int* ht,
                            int n, hipStream_t st) {
  std::vector<int> kinds;
  launch_t2N(t2, w.t2N, p.no, p.nv, st);
  if (p.prec != CC3_FP64) launch_lp_convert(t2, w.b, p.no, p.nv, w.lp, st);
  const bool lowp_contract = w.GbcX != nullptr;
  const int lpP = !lowp_contract || p.prec == CC3_FP32 ? 0 : p.prec == CC3_BF16X3 ? 2 : 3;
  if (lowp_contract && lpP == 0) {
    const int64_t gn = (int64_t)p.no * (p.nv + p.no) * p.nv * p.nv;
    launch_to_f32(w.b.Gbc, (float*)w.GbcX, gn, st);
    launch_to_f32(w.b.Gcb, (float*)w.GcbX, gn, st);
  } else if (lowp_contract) {
    launch_lp_contract_convert(w.b, p.prec, p.no, p.nv, w.GbcX, w.GcbX, st);
    for (int k = 0; k < 2; ++k)
      launch_lp_zero_pad(w.cubesX[k], (int64_t)p.batch * 4 * lpP * p.nv, p.nv, st);
  }
  // PLAN_CALLER_STREAM: every batch on the caller's stream, no runner streams or events
  const bool own = (p.flags & PLAN_CALLER_STREAM) != 0;
  if (!own) {
    HIPCHK(hipEventRecord(rn.ev_fork, st));
    for (int k = 0; k < NSTREAM; ++k) HIPCHK(hipStreamWaitEvent(rn.s[k], rn.ev_fork, 0));
  }
  // CC3_ONE_STREAM (or CC3_SERIAL=1 in the environment) keeps every batch on one stream;
  // so does a wide virtual space, where one batch's W build and Omega GEMM fill the
  // device for milliseconds each and the overlap measured slower (23/250/800: 4.94
  // against 5.06 s per call)
  static const int env_serial = env_int("CC3_SERIAL", 0);
  const int nstream =
      (own || env_serial || (p.flags & CC3_ONE_STREAM) || p.nv > 192) ? 1 : NSTREAM;
  const int ngroups = (n + p.batch - 1) / p.batch;
  for (int nbatch = 0; nbatch < ngroups; ++nbatch) {
    int t0, nb;
    batch_range(n, ngroups, nbatch, &t0, &nb);
    const int k = nbatch % nstream;
    hipStream_t sk = own ? st : rn.s[k];
    kinds.resize(nb);
    for (int t = 0; t < nb; ++t)
      kinds[t] = kind_of(ht[3 * (t0 + t)], ht[3 * (t0 + t) + 1], ht[3 * (t0 + t) + 2]);
    const int* tb = tri + 3 * t0;
    {
      Timer tm(pf, sk, FAM_W, wbuild_flops(p.no, p.nv, kinds.data(), nb), 0.0);
      if (p.prec == CC3_FP64)
        launch_wbuild(t2, w.t2N, w.b, tb, nb, w.cubes[k], p.no, p.nv, false, sk);
      else
        launch_wbuild_lp(w.lp, tb, nb, w.cubes[k], p.no, p.nv, false, sk);
    }
    {
      Timer tm(pf, sk, FAM_MIX, 0.0, 0.0);
      launch_mix(eps, tb, nb, w.cubes[k], lowp_contract && lpP == 0 ? (float*)w.cubesX[k] : nullptr,
                 lpP ? w.cubesX[k] : nullptr, lpP, p.no, p.nv, sk);
    }
    {
      Timer tm(pf, sk, FAM_OMEGA, omega_flops(p.no, p.nv, kinds.data(), nb), 0.0);
      if (lowp_contract && lpP == 0)
        launch_omega_f32((const float*)w.cubesX[k], (const float*)w.GbcX, (const float*)w.GcbX, tb,
                         nb, w.Pvv[k], p.no, p.nv, sk);
      else if (lowp_contract)
        launch_omega_lp(p.prec, w.cubesX[k], w.GbcX, w.GcbX, tb, nb, w.Pvv[k], p.no, p.nv, sk);
      else
        launch_omega(w.cubes[k], w.b, tb, nb, w.Pvv[k], p.no, p.nv, sk);
    }
    if (nbatch > 0 && !own) HIPCHK(hipStreamWaitEvent(sk, rn.ev_red[(nbatch - 1) % nstream], 0));
    {
      Timer tm(pf, sk, FAM_OMEGA_OO, omega_oo_flops(p.no, p.nv, kinds.data(), nb), 0.0);
      launch_omega_oo(w.cubes[k], w.b, tb, nb, w.OtT, p.no, p.nv, sk);
    }
    {
      Timer tm(pf, sk, FAM_REDUCE, 0.0, 0.0);
      launch_reduce(tb, nb, w.Pvv[k], w.Ot1, w.Ot2, p.no, p.nv, (p.flags & CC3_LOWP_CONTRACT) != 0,
                    sk);
    }
    if (!own) HIPCHK(hipEventRecord(rn.ev_red[k], sk));
  }
  if (!own) {
    for (int k = 0; k < NSTREAM; ++k) {
      HIPCHK(hipEventRecord(rn.ev_done[k], rn.s[k]));
      HIPCHK(hipStreamWaitEvent(st, rn.ev_done[k], 0));
    }
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

int residual_from_blocks(Runner& rn, Profiler* pf, const Plan& p, const Ws& w, const double* eps,
                         const double* t2, double* omega1, double* omega2, bool accumulate,
                         hipStream_t st, const double* omega2_in) {
  const int no = p.no, nv = p.nv;
  launch_fill(w.Ot1, (int64_t)no * nv, 0.0, st);
  launch_fill(w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
  launch_fill(w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
  launch_triple_table(w.tri, no, nbatches(p), st);
  std::vector<int> ht;
  host_triples(no, nbatches(p), ht);
  int rc = triple_loop(rn, pf, p, w, eps, t2, w.tri, ht.data(), p.ntri, st);
  if (rc) return rc;
  if (omega2_in)
    HIPCHK(hipMemcpyAsync(omega2, omega2_in, sizeof(double) * no * no * nv * nv,
                          hipMemcpyHostToDevice, st));
  {
    Timer tm(pf, st, FAM_BACK, 0.0, 0.0);
    launch_back_transform(w.Ot1, w.Ot2, w.OtT, omega1, omega2, no, nv, accumulate, st);
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

// Several requests in lockstep through packed launches: the per-request
// preparation, then step s runs batch s of every request that has one in the
// five packed launches of the triple loop, then the per-request back
// transformation.  Each request keeps its own plan, batches and reduction order,
// so its result is that of its own call.  host_jobs receives the job tables
// (they must outlive the copy into dev_jobs, which holds room for
// max_batches * ms.size() jobs).
int packed_residuals(const std::vector<PackMember>& ms, int prec, PackJob* dev_jobs,
                     std::vector<PackJob>& host_jobs, hipStream_t st) {
  const int nm = (int)ms.size();
  int nsteps = 0;
  for (const PackMember& m : ms) {
    const Plan& p = *m.p;
    const int no = p.no, nv = p.nv;
    int rc;
    if (m.rebuild && (rc = prepare_cholesky(nullptr, p, m.w, m.L, m.t1, st))) return rc;
    launch_fill(m.w.Ot1, (int64_t)no * nv, 0.0, st);
    launch_fill(m.w.Ot2, (int64_t)no * no * nv * nv, 0.0, st);
    launch_fill(m.w.OtT, (int64_t)no * no * nv * nv, 0.0, st);
    launch_triple_table(m.w.tri, no, nbatches(p), st);
    launch_t2N(m.t2, m.w.t2N, no, nv, st);
    if (prec != CC3_FP64) launch_lp_convert(m.t2, m.w.b, no, nv, m.w.lp, st);
    nsteps = std::max(nsteps, nbatches(p));
  }
  host_jobs.assign((size_t)nsteps * nm, PackJob{});
  std::vector<int> njobs(nsteps, 0);
  for (int s = 0; s < nsteps; ++s) {
    unsigned first[PK_N] = {0, 0, 0, 0, 0};
    for (const PackMember& m : ms) {
      const Plan& p = *m.p;
      const int nb_all = nbatches(p);
      if (s >= nb_all) continue;
      int t0, nb;
      batch_range(p.ntri, nb_all, s, &t0, &nb);
      PackJob j{};
      j.t2 = m.t2; j.t2N = m.w.t2N; j.eps = m.eps;
      j.Gw = m.w.b.Gw; j.Go = m.w.b.Go; j.Gbc = m.w.b.Gbc; j.Gcb = m.w.b.Gcb; j.Hs = m.w.b.Hs;
      j.lpt2 = m.w.lp.t2; j.lpt2N = m.w.lp.t2N; j.lpGwT = m.w.lp.GwT; j.lpGoT = m.w.lp.GoT;
      j.tri = m.w.tri + 3 * t0;
      j.cubes = m.w.cubes[0]; j.Pvv = m.w.Pvv[0];
      j.Ot1 = m.w.Ot1; j.Ot2 = m.w.Ot2; j.OtT = m.w.OtT;
      j.no = p.no; j.nv = p.nv; j.ntri = nb; j.nch = omega_kchunks(p.nv, nb);
      unsigned it[PK_N];
      pack_items(j, it);
      for (int k = 0; k < PK_N; ++k) { j.first[k] = first[k]; first[k] += it[k]; }
      host_jobs[(size_t)s * nm + njobs[s]++] = j;
    }
  }
  HIPCHK(hipMemcpyAsync(dev_jobs, host_jobs.data(), host_jobs.size() * sizeof(PackJob),
                        hipMemcpyHostToDevice, st));
  for (int s = 0; s < nsteps; ++s)
    launch_packed_step(dev_jobs + (size_t)s * nm, host_jobs.data() + (size_t)s * nm, njobs[s], prec,
                       st);
  for (const PackMember& m : ms)
    launch_back_transform(m.w.Ot1, m.w.Ot2, m.w.OtT, m.O1, m.O2, m.p->no, m.p->nv, false, st);
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

int pack_steps(const Plan& p) { return nbatches(p); }

// Algorithm 2 over every unordered triple: the same batched W build and mix as the
// residual, then per batch the Zo partials on the batch's stream and, chained in
// batch order, the Zo reduction and the output-stationary Zv contraction.
static int jacobian_prep_body(Runner& rn, Profiler* pf, const Plan& p, const Ws& w,
                              const double* eps, const double* t2, double* zv, double* zo,
                              bool accumulate, hipStream_t st);

int jacobian_prep_from_blocks(Runner& rn, Profiler* pf, const Plan& p, const Ws& w,
                              const double* eps, const double* t2, double* zv, double* zo,
                              bool accumulate, hipStream_t st) {
  int rc = rn.init();
  if (rc) return rc;
  rc = jacobian_prep_body(rn, pf, p, w, eps, t2, zv, zo, accumulate, st);
  if (rc) join_runner(rn, st);
  return rc;
}

static int jacobian_prep_body(Runner& rn, Profiler* pf, const Plan& p, const Ws& w,
                              const double* eps, const double* t2, double* zv, double* zo,
                              bool accumulate, hipStream_t st) {
  const int no = p.no, nv = p.nv;
  if (!accumulate) {
    launch_fill(zv, (int64_t)nv * nv * nv * no, 0.0, st);
    launch_fill(zo, (int64_t)nv * no * no * no, 0.0, st);
  }
  launch_triple_table(w.tri, no, nbatches(p), st);
  std::vector<int> ht, kinds;
  host_triples(no, nbatches(p), ht);
  launch_t2N(t2, w.t2N, no, nv, st);
  if (p.prec != CC3_FP64) launch_lp_convert(t2, w.b, no, nv, w.lp, st);
  HIPCHK(hipEventRecord(rn.ev_fork, st));
  for (int k = 0; k < NSTREAM; ++k) HIPCHK(hipStreamWaitEvent(rn.s[k], rn.ev_fork, 0));
  static const int env_serial = env_int("CC3_SERIAL", 0);
  // one stream from nv = 192 on, as in the residual loop
  const int nstream = (env_serial || (p.flags & CC3_ONE_STREAM) || p.nv > 192) ? 1 : NSTREAM;
  const int n = p.ntri;
  const int ngroups = nbatches(p);
  for (int nbatch = 0; nbatch < ngroups; ++nbatch) {
    int t0, nb;
    batch_range(n, ngroups, nbatch, &t0, &nb);
    const int k = nbatch % nstream;
    hipStream_t sk = rn.s[k];
    kinds.resize(nb);
    for (int t = 0; t < nb; ++t)
      kinds[t] = kind_of(ht[3 * (t0 + t)], ht[3 * (t0 + t) + 1], ht[3 * (t0 + t) + 2]);
    const int* tb = w.tri + 3 * t0;
    {
      Timer tm(pf, sk, FAM_W, wbuild_flops(no, nv, kinds.data(), nb), 0.0);
      if (p.prec == CC3_FP64)
        launch_wbuild(t2, w.t2N, w.b, tb, nb, w.cubes[k], no, nv, false, sk);
      else
        launch_wbuild_lp(w.lp, tb, nb, w.cubes[k], no, nv, false, sk);
    }
    {
      Timer tm(pf, sk, FAM_MIX, 0.0, 0.0);
      launch_mix(eps, tb, nb, w.cubes[k], nullptr, nullptr, 0, no, nv, sk);
    }
    {
      Timer tm(pf, sk, FAM_ZPREP, zprep_flops(no, nv, kinds.data(), nb) * ((double)no / (nv + no)), 0.0);
      launch_zo(w.cubes[k], w.b, tb, nb, w.Pvv[k], nullptr, no, nv, sk, false);
    }
    if (nbatch > 0) HIPCHK(hipStreamWaitEvent(sk, rn.ev_red[(nbatch - 1) % nstream], 0));
    {
      Timer tm(pf, sk, FAM_REDUCE, 0.0, 0.0);
      launch_zo(w.cubes[k], w.b, tb, nb, w.Pvv[k], zo, no, nv, sk, true);
    }
    {
      Timer tm(pf, sk, FAM_ZPREP, zprep_flops(no, nv, kinds.data(), nb) * ((double)nv / (nv + no)), 0.0);
      launch_zv(w.cubes[k], w.b, tb, nb, zv, no, nv, sk);
    }
    HIPCHK(hipEventRecord(rn.ev_red[k], sk));
  }
  for (int k = 0; k < NSTREAM; ++k) {
    HIPCHK(hipEventRecord(rn.ev_done[k], rn.s[k]));
    HIPCHK(hipStreamWaitEvent(st, rn.ev_done[k], 0));
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}

// CC3_CHECK: blocks the host until the input check has run.
int run_input_check(const Plan& p, const Ws& w, const double* eps, const double* L,
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

}  // namespace cc3
