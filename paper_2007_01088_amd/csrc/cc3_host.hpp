// Host-side core shared by the one-shot entry points (cc3_api.cpp) and the
// serving loop (cc3_server.cpp): error reporting, kernel timing, the
// two-stream runner, the workspace layout and the launch sequence of one
// residual evaluation.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "cc3.h"
#include "cc3_internal.hpp"

namespace cc3 {

// ---- errors ----------------------------------------------------------------
int fail(int code, const char* fmt, ...);
const char* last_error_str();  // this thread's last message
#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::cc3::fail(CC3_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int check_sizes(int no, int nv, int nchol, int prec);
int check_dev_ptr(const void* p, const char* what);
// Non-null check plus the memory kind: *host = false for device (or managed)
// memory, true for host memory, pageable or pinned.
int classify_ptr(const void* p, const char* what, bool* host);

// ---- kernel timing ------------------------------------------------------------
enum { FAM_T1 = 0, FAM_BUILD, FAM_W, FAM_MIX, FAM_OMEGA, FAM_REDUCE, FAM_BACK, FAM_ZPREP, FAM_OMEGA_OO,
       FAM_L3, FAM_DENSITY, NFAM };
extern const char* kFamilies[NFAM];

struct TimedLaunch {
  int family;
  hipEvent_t start, stop;
  double flops, bytes;
};

struct Profiler {
  bool on = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> pool;
  hipEvent_t take();
  void reset();
  int collect(cc3_kernel_stat* out, int max, int* count);
  void destroy();
};

// Brackets one launch with events when profiling is on (pf may be null).
struct Timer {
  Profiler* pf;
  hipStream_t st;
  TimedLaunch tl;
  bool on;
  Timer(Profiler* pf_, hipStream_t st_, int fam, double flops, double bytes);
  ~Timer();
};

// ---- two-stream runner --------------------------------------------------------
// The triple loop alternates its batches between two streams (each with its
// own cube and slab buffers), so that one batch's W build and mix overlap the
// previous batch's Omega contraction; the reductions into the residual are
// chained by events in batch order.
enum { NSTREAM = 2 };
struct Runner {
  bool ready = false;
  bool own0 = true;  // false: s[0] is the caller's stream
  hipStream_t s[NSTREAM];
  hipEvent_t ev_fork, ev_done[NSTREAM], ev_red[NSTREAM];
  // Creates the streams; with `s0` given, batches alternate between s0 and
  // one stream of the runner's own (fewer streams per concurrent request).
  int init(hipStream_t s0 = nullptr);
  void destroy();
};

// ---- workspace ----------------------------------------------------------------
struct Ws {
  Blocks b;
  CholeskyScratch cs;
  double *Ot1, *Ot2, *OtT, *t2N;
  double *cubes[2], *Pvv[2];
  // mixed-all (CC3_LOWP_CONTRACT) only, else null: low-precision Gbc and Gcb, and the
  // per-set views of tau~ (FP32 tau~ and tau~T, or the split-BF16 k-major views)
  void *GbcX, *GcbX, *cubesX[2];
  int* tri;
  int* flag;
  LpOperands lp;
  // one-shot calls: staging areas of host-memory eps, t1, t2, omega1 (null otherwise)
  double *st_eps, *st_t1, *st_t2, *st_o1;
};

// `with_blocks`: the integral blocks live in the workspace (one-shot calls) or
// elsewhere (resident per molecule, serving).  `cube_budget` bounds one cube
// buffer set in bytes (0: default).
int make_plan_ex(int no, int nv, int nchol, int prec, unsigned flags, bool with_blocks,
                 size_t cube_budget, Plan* p);
Ws carve(const Plan& p, void* ws, const Blocks* external_blocks);
size_t block_bytes(int no, int nv);
Blocks carve_blocks(int no, int nv, void* base);

// ---- launch sequences ---------------------------------------------------------
int prepare_cholesky(Profiler* pf, const Plan& p, const Ws& w, const double* L, const double* t1,
                     hipStream_t st);
int triple_loop(Runner& rn, Profiler* pf, const Plan& p, const Ws& w, const double* eps,
                const double* t2, const int* tri, const int* ht, int n, hipStream_t st);
// Ot <- 0, the whole restricted loop, back-transformation into (omega1, omega2).
// `omega2_in`, when given, is host memory copied into omega2 just before the
// back-transformation (CC3_ACCUMULATE into host outputs staged in t2N).
int residual_from_blocks(Runner& rn, Profiler* pf, const Plan& p, const Ws& w, const double* eps,
                         const double* t2, double* omega1, double* omega2, bool accumulate,
                         hipStream_t st, const double* omega2_in = nullptr);
// Algorithm 2: zv[a][b][i][d] = Z~v_{abid}, zo[a][j][i][l] = Z~o_{ajil} (zeroed first
// unless accumulate), over every unordered triple.
int jacobian_prep_from_blocks(Runner& rn, Profiler* pf, const Plan& p, const Ws& w,
                              const double* eps, const double* t2, double* zv, double* zo,
                              bool accumulate, hipStream_t st);
int run_input_check(const Plan& p, const Ws& w, const double* eps, const double* L,
                    const double* t2, hipStream_t st);

// One request of a packed group (serving): its plan and workspace, its inputs
// (device) and outputs, and whether its integral blocks are rebuilt first.
struct PackMember {
  const Plan* p;
  Ws w;
  const double *eps, *L, *t1, *t2;
  double *O1, *O2;
  bool rebuild;
};
int packed_residuals(const std::vector<PackMember>& ms, int prec, PackJob* dev_jobs,
                     std::vector<PackJob>& host_jobs, hipStream_t st);
int pack_steps(const Plan& p);  // batches of the plan (the pack's steps)

}  // namespace cc3

// A context of the one-shot calls: its device, kernel timing and runner streams.
struct cc3_ctx {
  int device;
  cc3::Profiler prof;
  cc3::Runner run;
  std::mutex mu;
};
