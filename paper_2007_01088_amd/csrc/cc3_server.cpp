// Serving entry points of the C ABI (include/cc3.h): a worker thread that
// admits residual requests from many resident molecules into a fixed device
// arena and runs them concurrently on independent stream slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cc3_host.hpp"

using namespace cc3;

namespace {

constexpr size_t NONE = ~(size_t)0;
constexpr int MAX_SLOTS = 8;

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

enum RState { R_QUEUED, R_RUNNING, R_DONE, R_FAILED, R_CANCELLED };

struct Molecule {
  int no, nv, nchol;
  size_t off = NONE, bytes = 0;
  double *eps, *L, *t1, *t2, *O1, *O2;
  int* flag;
  Blocks b;
  bool blocks_valid = false;
  uint64_t pending = 0;  // ticket of the request not yet collected (0: none)
};

struct Request {
  uint64_t mol;
  int prec;
  unsigned flags;
  bool rebuild;
  int state = R_QUEUED;
  int rc = CC3_OK;
  std::string msg;
  Plan plan;
  size_t off = NONE;
  int slot = -1;
  cc3_timing tm{};
};

struct Slot {
  bool busy = false;
  uint64_t ticket = 0;
  std::vector<uint64_t> pack;      // the requests of a packed group (empty: one request)
  std::vector<PackJob> pack_jobs;  // host copy of the group's job tables
  size_t pack_off = ~(size_t)0, pack_bytes = 0;  // arena region of the device job tables
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  Runner rn;
};

// First-fit allocator over [0, size) in 256-byte units.
struct Arena {
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> holes;  // offset -> length
  void init(size_t n) { size = n; holes.clear(); holes[0] = n; }
  size_t alloc(size_t n) {
    n = round256(n);
    for (auto it = holes.begin(); it != holes.end(); ++it) {
      if (it->second < n) continue;
      const size_t at = it->first, len = it->second;
      holes.erase(it);
      if (len > n) holes[at + n] = len - n;
      used += n;
      peak = std::max(peak, used);
      return at;
    }
    return NONE;
  }
  void release(size_t at, size_t n) {
    n = round256(n);
    used -= n;
    auto it = holes.emplace(at, n).first;
    auto nx = std::next(it);
    if (nx != holes.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      holes.erase(nx);
    }
    if (it != holes.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        holes.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& h : holes) m = std::max(m, h.second);
    return m;
  }
};

size_t molecule_bytes(int no, int nv, int nchol) {
  const size_t o = no, v = nv, n = no + nv;
  return round256(n * 8) + round256((size_t)nchol * n * n * 8) + round256(o * v * 8) * 2 +
         round256(o * o * v * v * 8) * 2 + block_bytes(no, nv) + 256;
}

bool is_device(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// A device pointer must address `bytes` inside one allocation; a host pointer
// is taken as given.
int check_span(const void* p, size_t bytes, const char* what) {
  if (!p) return fail(CC3_E_INVAL, "%s is NULL", what);
  if (!is_device(p)) return CC3_OK;
  void* base = nullptr;
  size_t len = 0;
  if (hipMemGetAddressRange(&base, &len, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return CC3_OK;
  }
  if ((const char*)p + bytes > (const char*)base + len)
    return fail(CC3_E_INVAL, "%s: %zu bytes run past the end of its allocation", what, bytes);
  return CC3_OK;
}

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct cc3_server {
  int device = 0;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int nslots = 1;
  size_t cube_budget = 0;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  Arena al;
  std::unordered_map<uint64_t, Molecule> mols;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> fifo;
  Slot slots[MAX_SLOTS];
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  int64_t n_sub = 0, n_done = 0, n_fail = 0, n_cancel = 0, n_packed = 0, n_packs = 0;
  int inflight = 0, max_seen = 0;
  // packing: at most max_pack requests of at most pack_flops nominal FLOP each share
  // the launches of one slot (max_pack 1: no packing)
  int max_pack = 8;
  double pack_flops = 2e12;

  // host <-> arena copies of the calling threads
  std::mutex up_mu;
  hipStream_t up = nullptr;
  hipEvent_t ev_ref = nullptr;  // device-clock origin for start_s
  double ref_s = 0.0;

  void run();
  void finish(uint64_t ticket, int rc, const char* msg);
  void finish_one(uint64_t ticket, Slot& s, int rc, const char* msg);
  int launch(uint64_t ticket, Request& r, Molecule& m, Slot& s);
  int launch_pack(Slot& s, const std::vector<PackMember>& ms, int prec);
  int ensure_slot(Slot& s);
  bool packable(const Request& r) const;
};

// ---------------------------------------------------------------------------
// worker
// ---------------------------------------------------------------------------
// Completion of the request(s) on the slot of `ticket`: every request of a packed
// group finishes with the group.
void cc3_server::finish(uint64_t ticket, int rc, const char* msg) {
  Slot& s = slots[reqs[ticket].slot];
  if (s.pack.empty()) {
    finish_one(ticket, s, rc, msg);
  } else {
    for (uint64_t t : s.pack) finish_one(t, s, rc, msg);
    s.pack.clear();
    if (s.pack_off != NONE) al.release(s.pack_off, s.pack_bytes);
    s.pack_off = NONE;
  }
  s.busy = false;
  s.ticket = 0;
}

void cc3_server::finish_one(uint64_t ticket, Slot& s, int rc, const char* msg) {
  Request& r = reqs[ticket];
  if (rc == CC3_OK) {
    float ms = 0.f, st = 0.f;
    if (hipEventElapsedTime(&ms, s.ev0, s.ev1) == hipSuccess) r.tm.device_ms = ms;
    if (hipEventElapsedTime(&st, ev_ref, s.ev0) == hipSuccess) r.tm.start_s = ref_s + st * 1e-3;
    (void)hipGetLastError();
  }
  r.tm.finish_s = now_s(t0);
  r.rc = rc;
  r.state = rc == CC3_OK ? R_DONE : R_FAILED;
  if (msg) r.msg = msg;
  if (rc != CC3_OK) {
    mols[r.mol].blocks_valid = false;
    ++n_fail;
  } else {
    ++n_done;
  }
  al.release(r.off, r.plan.total);
  r.off = NONE;
  --inflight;
}

int cc3_server::ensure_slot(Slot& s) {
  HIPCHK(hipSetDevice(device));
  if (!s.st) {
    HIPCHK(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&s.ev0));
    HIPCHK(hipEventCreate(&s.ev1));
    int rc0 = s.rn.init(s.st);  // the slot's stream carries every other batch
    if (rc0) return rc0;
  }
  return CC3_OK;
}

// A request may join a packed group: a W-only precision, and small enough that
// its own launches would leave the device partly idle.
bool cc3_server::packable(const Request& r) const {
  if (max_pack < 2) return false;
  const double v = r.plan.nv, o = r.plan.no;
  return 4.0 * v * v * v * v * o * o * o <= pack_flops;
}

// The members of slot s's packed group (with the lock held).
static std::vector<PackMember> pack_members(cc3_server& sv, const Slot& s, int* prec) {
  std::vector<PackMember> ms;
  for (uint64_t t : s.pack) {
    Request& r = sv.reqs.at(t);
    Molecule& m = sv.mols.at(r.mol);
    PackMember pm;
    pm.p = &r.plan;
    pm.w = carve(r.plan, sv.arena + r.off, &m.b);
    pm.eps = m.eps; pm.L = m.L; pm.t1 = m.t1; pm.t2 = m.t2;
    pm.O1 = m.O1; pm.O2 = m.O2;
    pm.rebuild = r.rebuild;
    *prec = r.prec;
    ms.push_back(pm);
  }
  return ms;
}

// Enqueues a packed group on slot s (called without the lock held; the group's
// requests, molecules and the slot are reserved for this thread; ms was built
// under the lock).
int cc3_server::launch_pack(Slot& s, const std::vector<PackMember>& ms, int prec) {
  int rc = ensure_slot(s);
  if (rc) return rc;
  HIPCHK(hipEventRecord(s.ev0, s.st));
  if ((rc = packed_residuals(ms, prec, (PackJob*)(arena + s.pack_off), s.pack_jobs, s.st)))
    return rc;
  HIPCHK(hipEventRecord(s.ev1, s.st));
  return CC3_OK;
}

// Enqueues the whole request on slot s (called without the lock held: the
// request, its molecule and the slot are reserved for this thread).
int cc3_server::launch(uint64_t, Request& r, Molecule& m, Slot& s) {
  int rc0 = ensure_slot(s);
  if (rc0) return rc0;
  const Plan& p = r.plan;
  Ws w = carve(p, arena + r.off, &m.b);
  HIPCHK(hipEventRecord(s.ev0, s.st));
  int rc;
  if (r.rebuild && (rc = prepare_cholesky(nullptr, p, w, m.L, m.t1, s.st))) return rc;
  if ((rc = residual_from_blocks(s.rn, nullptr, p, w, m.eps, m.t2, m.O1, m.O2, false, s.st)))
    return rc;
  HIPCHK(hipEventRecord(s.ev1, s.st));
  return CC3_OK;
}

void cc3_server::run() {
  if (hipSetDevice(device) != hipSuccess) return;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // completions
    for (int k = 0; k < nslots; ++k) {
      Slot& s = slots[k];
      if (!s.busy || reqs[s.ticket].state != R_RUNNING) continue;
      hipError_t q = hipEventQuery(s.ev1);
      if (q == hipSuccess) {
        finish(s.ticket, CC3_OK, nullptr);
        cv_done.notify_all();
      } else if (q != hipErrorNotReady) {
        (void)hipGetLastError();
        finish(s.ticket, CC3_E_DEVICE, hipGetErrorString(q));
        cv_done.notify_all();
      }
    }
    // admissions, in arrival order
    while (!fifo.empty()) {
      int k = 0;
      while (k < nslots && slots[k].busy) ++k;
      if (k == nslots) break;
      const uint64_t t = fifo.front();
      Request& r = reqs[t];
      const size_t off = al.alloc(r.plan.total);
      if (off == NONE) {
        if (inflight > 0) break;  // wait for memory to come back
        fifo.pop_front();
        r.state = R_FAILED;
        r.rc = CC3_E_NOMEM;
        char buf[160];
        snprintf(buf, sizeof buf,
                 "request needs %zu arena bytes; the largest free hole is %zu with nothing in flight",
                 r.plan.total, al.largest());
        r.msg = buf;
        r.tm.admit_s = r.tm.finish_s = now_s(t0);
        ++n_fail;
        cv_done.notify_all();
        continue;
      }
      fifo.pop_front();
      Slot& s = slots[k];
      s.busy = true;
      s.ticket = t;
      r.off = off;
      // packing: the following small requests of the same precision join this one,
      // as long as their workspaces and the group's job tables fit in the arena
      s.pack.clear();
      if (packable(r)) {
        s.pack.push_back(t);
        int steps = pack_steps(r.plan);
        while ((int)s.pack.size() < max_pack && !fifo.empty()) {
          Request& q = reqs[fifo.front()];
          if (!packable(q) || q.prec != r.prec) break;
          const size_t qoff = al.alloc(q.plan.total);
          if (qoff == NONE) break;
          q.off = qoff;
          s.pack.push_back(fifo.front());
          fifo.pop_front();
          steps = std::max(steps, pack_steps(q.plan));
        }
        s.pack_bytes = (size_t)steps * s.pack.size() * sizeof(PackJob);
        s.pack_off = s.pack.size() > 1 ? al.alloc(s.pack_bytes) : NONE;
        if (s.pack_off == NONE) {  // no group: the others go back to the queue front
          for (size_t g = s.pack.size(); g-- > 1;) {
            Request& q = reqs[s.pack[g]];
            al.release(q.off, q.plan.total);
            q.off = NONE;
            fifo.push_front(s.pack[g]);
          }
          s.pack.clear();
        }
      }
      std::vector<uint64_t> group = s.pack.empty() ? std::vector<uint64_t>{t} : s.pack;
      for (uint64_t gt : group) {
        Request& q = reqs[gt];
        q.slot = k;
        q.tm.slot = k;
        q.tm.rebuilt = q.rebuild ? 1 : 0;
        q.tm.admit_s = now_s(t0);
        q.state = R_RUNNING;  // from here on cc3_cancel leaves it alone
        ++inflight;
      }
      if (group.size() > 1) {
        n_packed += (int64_t)group.size();
        ++n_packs;
      }
      max_seen = std::max(max_seen, inflight);
      Molecule& m = mols[r.mol];
      int pprec = CC3_FP64;
      const std::vector<PackMember> ms =
          s.pack.empty() ? std::vector<PackMember>() : pack_members(*this, s, &pprec);
      lk.unlock();
      const int rc = s.pack.empty() ? launch(t, r, m, s) : launch_pack(s, ms, pprec);
      std::string err = rc ? last_error_str() : std::string();
      lk.lock();
      if (rc) {
        // the failed enqueue may have left work on the slot's streams: drain it
        // before the workspace goes back to the arena
        if (s.st) (void)hipStreamSynchronize(s.st);
        for (int q = 0; q < NSTREAM; ++q)
          if (s.rn.ready && s.rn.s[q]) (void)hipStreamSynchronize(s.rn.s[q]);
        (void)hipGetLastError();
        finish(t, rc, err.c_str());
        cv_done.notify_all();
      }
    }
    if (stop && inflight == 0 && fifo.empty()) break;
    if (inflight > 0)
      cv_work.wait_for(lk, std::chrono::microseconds(50));
    else
      cv_work.wait(lk, [&] { return stop || !fifo.empty(); });
  }
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" int cc3_server_create(cc3_server** out, int device, void* arena, size_t arena_bytes,
                                 int max_inflight) {
  if (!out) return fail(CC3_E_INVAL, "cc3_server_create: out is NULL");
  if (max_inflight < 1 || max_inflight > MAX_SLOTS)
    return fail(CC3_E_INVAL, "max_inflight must be in [1, %d] (got %d)", MAX_SLOTS, max_inflight);
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n)
    return fail(CC3_E_INVAL, "device %d out of range (%d devices)", device, n);
  HIPCHK(hipSetDevice(device));
  if (!arena) return fail(CC3_E_INVAL, "arena is NULL");
  if (((uintptr_t)arena) & 255) return fail(CC3_E_INVAL, "arena must be 256-byte aligned");
  int rc = check_dev_ptr(arena, "arena");
  if (rc) return rc;
  if ((rc = check_span(arena, arena_bytes, "arena"))) return rc;
  cc3_server* s = new cc3_server();
  s->device = device;
  s->arena = (char*)arena;
  s->arena_bytes = arena_bytes & ~(size_t)255;
  s->nslots = max_inflight;
  // one cube buffer set per request: large enough for full-size batches,
  // small enough that every slot can hold a request
  s->cube_budget = std::min<size_t>((size_t)4096 << 20,
                                    std::max<size_t>((size_t)128 << 20,
                                                     s->arena_bytes / (8 * (size_t)max_inflight)));
  s->al.init(s->arena_bytes);
  s->t0 = std::chrono::steady_clock::now();
  if (hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&s->ev_ref) != hipSuccess) {
    delete s;
    return fail(CC3_E_DEVICE, "could not create the server's stream");
  }
  if (hipEventRecord(s->ev_ref, s->up) != hipSuccess ||
      hipEventSynchronize(s->ev_ref) != hipSuccess) {
    hipStreamDestroy(s->up);
    hipEventDestroy(s->ev_ref);
    delete s;
    return fail(CC3_E_DEVICE, "could not start the server's clock");
  }
  s->ref_s = now_s(s->t0);
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return CC3_OK;
}

extern "C" int cc3_server_destroy(cc3_server* s) {
  if (!s) return CC3_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (uint64_t t : s->fifo) {
      Request& r = s->reqs[t];
      r.state = R_CANCELLED;
      r.rc = CC3_E_CANCELLED;
      ++s->n_cancel;
    }
    s->fifo.clear();
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  if (s->worker.joinable()) s->worker.join();
  hipSetDevice(s->device);
  for (int k = 0; k < MAX_SLOTS; ++k) {
    Slot& sl = s->slots[k];
    if (sl.st) {
      hipStreamSynchronize(sl.st);
      hipStreamDestroy(sl.st);
      hipEventDestroy(sl.ev0);
      hipEventDestroy(sl.ev1);
    }
    sl.rn.destroy();
  }
  hipStreamDestroy(s->up);
  hipEventDestroy(s->ev_ref);
  delete s;
  return CC3_OK;
}

static int request_plan(const cc3_server* s, int no, int nv, int nchol, int prec, unsigned flags,
                        Plan* p) {
  int rc = check_sizes(no, nv, nchol, prec);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1");
  make_plan_ex(no, nv, nchol, prec, flags, false, s->cube_budget, p);
  return CC3_OK;
}

extern "C" int cc3_server_footprint(cc3_server* s, int no, int nv, int nchol, int prec,
                                    size_t* resident, size_t* transient) {
  if (!s) return fail(CC3_E_INVAL, "server is NULL");
  Plan p;
  int rc = request_plan(s, no, nv, nchol, prec, 0, &p);
  if (rc) return rc;
  if (resident) *resident = round256(molecule_bytes(no, nv, nchol));
  if (transient) *transient = round256(p.total);
  return CC3_OK;
}

extern "C" int cc3_molecule_register(cc3_server* s, int no, int nv, int nchol, const double* eps,
                                     const double* L, const double* t1, uint64_t* mol) {
  if (!s || !mol) return fail(CC3_E_INVAL, "cc3_molecule_register: server or mol is NULL");
  Plan p;
  int rc = request_plan(s, no, nv, nchol, CC3_FP64, 0, &p);
  if (rc) return rc;
  const size_t n = no + nv;
  if ((rc = check_span(eps, n * 8, "eps")) || (rc = check_span(L, (size_t)nchol * n * n * 8, "L")))
    return rc;
  if (t1 && (rc = check_span(t1, (size_t)no * nv * 8, "t1"))) return rc;
  Molecule m;
  m.no = no; m.nv = nv; m.nchol = nchol;
  m.bytes = molecule_bytes(no, nv, nchol);
  {
    std::lock_guard<std::mutex> g(s->mu);
    m.off = s->al.alloc(m.bytes);
    if (m.off == NONE)
      return fail(CC3_E_NOMEM, "molecule needs %zu arena bytes; the largest free hole is %zu",
                  m.bytes, s->al.largest());
  }
  const size_t o = no, v = nv;
  char* c = s->arena + m.off;
  auto take = [&](size_t bytes) { char* at = c; c += round256(bytes); return at; };
  m.eps = (double*)take(n * 8);
  m.L = (double*)take((size_t)nchol * n * n * 8);
  m.t1 = (double*)take(o * v * 8);
  m.O1 = (double*)take(o * v * 8);
  m.t2 = (double*)take(o * o * v * v * 8);
  m.O2 = (double*)take(o * o * v * v * 8);
  m.b = carve_blocks(no, nv, take(block_bytes(no, nv)));
  m.flag = (int*)take(256);
  {
    std::lock_guard<std::mutex> g(s->up_mu);
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipMemcpyAsync(m.eps, eps, n * 8, hipMemcpyDefault, s->up);
    if (e == hipSuccess)
      e = hipMemcpyAsync(m.L, L, (size_t)nchol * n * n * 8, hipMemcpyDefault, s->up);
    if (e == hipSuccess) {
      if (t1) e = hipMemcpyAsync(m.t1, t1, o * v * 8, hipMemcpyDefault, s->up);
      else launch_fill(m.t1, (int64_t)(o * v), 0.0, s->up);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->up);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      std::lock_guard<std::mutex> g2(s->mu);
      s->al.release(m.off, m.bytes);
      return fail(CC3_E_DEVICE, "molecule input copy failed: %s", hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> g(s->mu);
  const uint64_t id = s->next_id++;
  s->mols.emplace(id, m);
  *mol = id;
  return CC3_OK;
}

extern "C" int cc3_molecule_release(cc3_server* s, uint64_t mol) {
  if (!s) return fail(CC3_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->mols.find(mol);
  if (it == s->mols.end()) return fail(CC3_E_NOTFOUND, "unknown molecule %llu",
                                       (unsigned long long)mol);
  if (it->second.pending)
    return fail(CC3_E_BUSY, "molecule %llu has an uncollected request",
                (unsigned long long)mol);
  s->al.release(it->second.off, it->second.bytes);
  s->mols.erase(it);
  return CC3_OK;
}

extern "C" int cc3_submit(cc3_server* s, uint64_t mol, const double* t1, const double* t2,
                          int prec, unsigned flags, uint64_t* ticket) {
  if (!s || !ticket) return fail(CC3_E_INVAL, "cc3_submit: server or ticket is NULL");
  if (flags & ~(unsigned)(CC3_ACCUMULATE | CC3_CHECK | CC3_DETERMINISTIC))
    return fail(CC3_E_INVAL, "cc3_submit takes CC3_ACCUMULATE, CC3_CHECK and CC3_DETERMINISTIC "
                "only (flags 0x%x)", flags);
  Molecule* m;
  Plan p;
  uint64_t t;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(CC3_E_INVAL, "server is shutting down");
    auto it = s->mols.find(mol);
    if (it == s->mols.end())
      return fail(CC3_E_NOTFOUND, "unknown molecule %llu", (unsigned long long)mol);
    m = &it->second;
    if (m->pending)
      return fail(CC3_E_BUSY, "molecule %llu has an uncollected request",
                  (unsigned long long)mol);
    int rc = request_plan(s, m->no, m->nv, m->nchol, prec, flags, &p);
    if (rc) return rc;
    if (p.total > s->arena_bytes)
      return fail(CC3_E_NOMEM, "request needs %zu arena bytes, the arena has %zu", p.total,
                  s->arena_bytes);
    t = s->next_id++;
    m->pending = t;  // reserves the molecule's buffers for this thread
  }
  const size_t o = m->no, v = m->nv;
  int rc = check_span(t2, o * o * v * v * 8, "t2");
  if (!rc && t1) rc = check_span(t1, o * v * 8, "t1");
  const double arrival = now_s(s->t0);
  if (!rc) {
    std::lock_guard<std::mutex> g(s->up_mu);
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipMemcpyAsync(m->t2, t2, o * o * v * v * 8, hipMemcpyDefault, s->up);
    if (e == hipSuccess && t1) e = hipMemcpyAsync(m->t1, t1, o * v * 8, hipMemcpyDefault, s->up);
    if (e == hipSuccess) e = hipStreamSynchronize(s->up);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      rc = fail(CC3_E_DEVICE, "request input copy failed: %s", hipGetErrorString(e));
    } else if (flags & CC3_CHECK) {
      Ws w{};
      w.flag = m->flag;
      rc = run_input_check(p, w, m->eps, m->L, m->t2, s->up);
    }
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (rc) {
    if (t1) m->blocks_valid = false;
    m->pending = 0;
    return rc;
  }
  Request r;
  r.mol = mol;
  r.prec = prec;
  r.flags = flags;
  r.rebuild = (t1 != nullptr) || !m->blocks_valid;
  r.plan = p;
  r.tm.arrival_s = arrival;
  r.tm.slot = -1;
  m->blocks_valid = true;  // once this request has run (reset if it fails)
  s->reqs.emplace(t, r);
  s->fifo.push_back(t);
  ++s->n_sub;
  *ticket = t;
  s->cv_work.notify_all();
  return CC3_OK;
}

extern "C" int cc3_poll(cc3_server* s, uint64_t ticket, int* done) {
  if (!s || !done) return fail(CC3_E_INVAL, "cc3_poll: server or done is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end())
    return fail(CC3_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  const int st = it->second.state;
  *done = (st == R_DONE || st == R_FAILED || st == R_CANCELLED) ? 1 : 0;
  return CC3_OK;
}

extern "C" int cc3_wait(cc3_server* s, uint64_t ticket, double* omega1, double* omega2,
                        cc3_timing* timing) {
  if (!s) return fail(CC3_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end())
    return fail(CC3_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = &it->second;
  s->cv_done.wait(lk, [&] {
    return r->state == R_DONE || r->state == R_FAILED || r->state == R_CANCELLED;
  });
  Molecule& m = s->mols[r->mol];
  int rc = r->rc;
  std::string msg = r->msg;
  if (timing) *timing = r->tm;
  const bool acc = (r->flags & CC3_ACCUMULATE) != 0;
  if (rc == CC3_OK && (omega1 || omega2)) {
    // the molecule's result stays put until the ticket is collected below
    lk.unlock();
    const size_t n1 = (size_t)m.no * m.nv, n2 = n1 * m.no * m.nv;
    if (acc && ((omega1 && !is_device(omega1)) || (omega2 && !is_device(omega2)))) {
      rc = fail(CC3_E_INVAL, "CC3_ACCUMULATE needs device outputs");
    } else if ((omega1 && (rc = check_span(omega1, n1 * 8, "omega1"))) ||
               (omega2 && (rc = check_span(omega2, n2 * 8, "omega2")))) {
    } else {
      std::lock_guard<std::mutex> g(s->up_mu);
      hipError_t e = hipSetDevice(s->device);
      if (acc) {
        if (omega1) launch_add(omega1, m.O1, (int64_t)n1, s->up);
        if (omega2) launch_add(omega2, m.O2, (int64_t)n2, s->up);
        if (e == hipSuccess) e = hipGetLastError();
      } else {
        if (e == hipSuccess && omega1)
          e = hipMemcpyAsync(omega1, m.O1, n1 * 8, hipMemcpyDefault, s->up);
        if (e == hipSuccess && omega2)
          e = hipMemcpyAsync(omega2, m.O2, n2 * 8, hipMemcpyDefault, s->up);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(s->up);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(CC3_E_DEVICE, "result copy failed: %s", hipGetErrorString(e));
      }
    }
    lk.lock();
  } else if (rc != CC3_OK) {
    fail(rc, "%s", msg.empty() ? "request failed" : msg.c_str());
  }
  m.pending = 0;
  s->reqs.erase(ticket);
  return rc;
}

extern "C" int cc3_cancel(cc3_server* s, uint64_t ticket) {
  if (!s) return fail(CC3_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end())
    return fail(CC3_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request& r = it->second;
  if (r.state != R_QUEUED) return fail(CC3_E_BUSY, "ticket %llu was already admitted",
                                       (unsigned long long)ticket);
  auto q = std::find(s->fifo.begin(), s->fifo.end(), ticket);
  if (q != s->fifo.end()) s->fifo.erase(q);
  r.state = R_CANCELLED;
  r.rc = CC3_E_CANCELLED;
  r.msg = "cancelled";
  if (r.rebuild) s->mols[r.mol].blocks_valid = false;
  ++s->n_cancel;
  s->cv_done.notify_all();
  return CC3_OK;
}

extern "C" int cc3_server_get_stats(cc3_server* s, cc3_server_stats* out) {
  if (!s || !out) return fail(CC3_E_INVAL, "cc3_server_get_stats: bad argument");
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->n_sub;
  out->completed = s->n_done;
  out->failed = s->n_fail;
  out->cancelled = s->n_cancel;
  out->queued = (int)s->fifo.size();
  out->inflight = s->inflight;
  out->max_inflight_seen = s->max_seen;
  out->molecules = (int)s->mols.size();
  out->arena_bytes = s->arena_bytes;
  out->arena_used = s->al.used;
  out->arena_peak = s->al.peak;
  out->packed = s->n_packed;
  out->packs = s->n_packs;
  return CC3_OK;
}

extern "C" int cc3_server_set_packing(cc3_server* s, int max_pack, double max_request_flops) {
  if (!s) return fail(CC3_E_INVAL, "server is NULL");
  if (max_pack < 1 || max_pack > 64 || !(max_request_flops >= 0.0))
    return fail(CC3_E_INVAL, "max_pack must be in [1, 64] and max_request_flops >= 0");
  std::lock_guard<std::mutex> g(s->mu);
  s->max_pack = max_pack;
  s->pack_flops = max_request_flops;
  return CC3_OK;
}
