// The transition-density loop (Algorithm 3, the triples contributions to
// D^{m,0}) on the caller's stream: workspace plan, the loop over occupied pairs,
// and its C-ABI entry points.
//
// Each pair (i, j), i >= j, is one batch holding the ordered triples (i, j, k)
// for every k: their t3 (W build, mix) and left-state L3 (the same engine with
// the L3 operands, the mix with the outer products and the (omega - eps)
// denominator), then the contractions of kern_density.hip.  Each unordered
// triple is sorted in exactly one pair and contributes its D_cd, Y^o and D_kc
// terms there; every pair contributes its Gram matrix to D_lk.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "cc3_density.hpp"
#include "cc3_host.hpp"

using namespace cc3;

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct DPlan {
  int no, nv, nchol, npairs, ntask;
  size_t cube;  // doubles per cube (cube_slot: nv x nv rows at the padded pitch)
  size_t off_Gw, off_Gl, off_Go, off_Go3, off_Jo, off_F, off_t2N, off_l2M, off_Y;
  size_t off_part, off_py, off_pkc, off_tri, off_task, off_cubes;
  size_t part_doubles, py_doubles, pkc_doubles, chol_bytes;
  size_t total;
  std::vector<int> htri;             // [pair][k][3]
  std::vector<int> htask;            // [task][D3_TASK_INTS]
  std::vector<int> task0, ntasks;    // per pair
  std::vector<int> pi, pj;           // the pair's (i, j)
};

// The distinct orderings of (i, j, k) in the order of itertools.permutations.
const int kPermH[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

void make_dplan(int no, int nv, int nchol, DPlan* p) {
  const size_t o = no, v = nv, J = nchol;
  p->no = no; p->nv = nv; p->nchol = nchol;
  p->cube = (size_t)cube_slot(nv);  // one padded cube
  p->npairs = no * (no + 1) / 2;
  p->htri.clear(); p->htask.clear(); p->task0.clear(); p->ntasks.clear(); p->pi.clear();
  p->pj.clear();
  for (int i = 0; i < no; ++i)
    for (int j = 0; j <= i; ++j) {
      p->pi.push_back(i);
      p->pj.push_back(j);
      for (int k = 0; k < no; ++k) {
        p->htri.push_back(i); p->htri.push_back(j); p->htri.push_back(k);
      }
      p->task0.push_back((int)p->htask.size() / D3_TASK_INTS);
      const int nown = (i == j) ? j : j + 1;
      int nt = 0;
      for (int k = 0; k < nown; ++k) {
        const int tr[3] = {i, j, k};
        for (int oi = 0; oi < 6; ++oi) {
          const int pp = tr[kPermH[oi][0]], qq = tr[kPermH[oi][1]], rr = tr[kPermH[oi][2]];
          bool dup = false;
          for (int o2 = 0; o2 < oi; ++o2)
            dup = dup || (tr[kPermH[o2][0]] == pp && tr[kPermH[o2][1]] == qq &&
                          tr[kPermH[o2][2]] == rr);
          if (dup) continue;
          const int e[D3_TASK_INTS] = {k, oi, pp, qq, rr};
          p->htask.insert(p->htask.end(), e, e + D3_TASK_INTS);
          ++nt;
        }
      }
      p->ntasks.push_back(nt);
    }
  p->ntask = (int)p->htask.size() / D3_TASK_INTS;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off = a256(off + bytes); return at; };
  p->off_Gw = take(o * v * v * v * 8);
  p->off_Gl = take(o * v * v * v * 8);
  p->off_Go = take(o * o * o * v * 8);
  p->off_Go3 = take(o * o * o * v * 8);
  p->off_Jo = take(o * o * v * v * 8);
  p->off_F = take(o * v * 8);
  p->off_t2N = take(o * o * v * v * 8);
  p->off_l2M = take(o * o * v * v * 8);
  p->off_Y = take(o * o * o * v * 8);
  // partial slabs: D_cd, Gram and D_ld share one region; Y^o and D_kc have their own
  size_t cd = 0, vy = 0, vk = 0;
  for (int nown = 1; nown <= no; ++nown)
    cd = std::max(cd, (size_t)nown * 3 * d3_cd_chunks(nv, nown) * v * v);
  int maxt = 1;
  for (int x : p->ntasks) maxt = std::max(maxt, x);
  for (int nt = 1; nt <= maxt; ++nt) {
    vy = std::max(vy, (size_t)nt * d3_vec_chunks(nv, nt, no) * v * o);
    vk = std::max(vk, (size_t)nt * d3_vec_chunks(nv, nt, 1) * v);
  }
  const size_t gr = (size_t)d3_gram_chunks(nv, no) * o * o;
  const size_t ld = (size_t)d3_ld_chunks(no, nv) * o * v;
  p->part_doubles = std::max(std::max(cd, gr), ld);
  p->py_doubles = vy;
  p->pkc_doubles = vk;
  p->off_part = take(p->part_doubles * 8);
  p->off_py = take(vy * 8);
  p->off_pkc = take(vk * 8);
  p->off_tri = take(p->htri.size() * sizeof(int));
  p->off_task = take(std::max<size_t>(1, p->htask.size()) * sizeof(int));
  // the Cholesky scratch and the build's temporary (vv|ov) block share the cube region
  p->chol_bytes = a256(J * v * v * 8) + a256(J * o * o * 8) * 2 + a256(J * o * v * 8) * 2 +
                  a256(J * 8) + a256(J * o * o * 8);
  const size_t cubes = a256((size_t)D3_NSLOT * o * p->cube * 8);
  p->off_cubes = take(std::max(cubes, p->chol_bytes + a256(o * v * v * v * 8)));
  p->total = off;
}

int check_density_sizes(int no, int nv, int nchol) {
  int rc = check_sizes(no, nv, nchol, CC3_FP64);
  if (rc) return rc;
  if (nchol < 1) return fail(CC3_E_INVAL, "nchol must be >= 1 (got %d)", nchol);
  if (nv > 400)
    return fail(CC3_E_INVAL, "the transition-density loop supports nv <= 400 (got %d)", nv);
  return CC3_OK;
}

}  // namespace

extern "C" int cc3_transition_density_workspace_size(int no, int nv, int nchol, size_t* bytes) {
  if (!bytes) return fail(CC3_E_INVAL, "cc3_transition_density_workspace_size: bytes is NULL");
  int rc = check_density_sizes(no, nv, nchol);
  if (rc) return rc;
  DPlan p;
  make_dplan(no, nv, nchol, &p);
  *bytes = p.total;
  return CC3_OK;
}

extern "C" int cc3_transition_density(cc3_ctx* c, int no, int nv, int nchol, const double* eps,
                                      const double* L, const double* t1, const double* t2,
                                      const double* l1, const double* l2, double omega,
                                      double* D_cd, double* D_kc, double* D_ld, double* D_lk,
                                      double* Yo, unsigned flags, void* ws, size_t ws_bytes,
                                      cc3_stream_t stream) {
  if (!c) return fail(CC3_E_INVAL, "ctx is NULL");
  int rc = check_density_sizes(no, nv, nchol);
  if (rc) return rc;
  if (flags & ~(unsigned)(CC3_ACCUMULATE | CC3_DETERMINISTIC))
    return fail(CC3_E_INVAL, "flags 0x%x: cc3_transition_density accepts CC3_ACCUMULATE and "
                "CC3_DETERMINISTIC", flags);
  HIPCHK(hipSetDevice(c->device));
  const void* ptrs[] = {eps, L, t1, t2, l1, l2, D_cd, D_kc, D_ld, D_lk, ws};
  const char* names[] = {"eps", "L", "t1", "t2", "l1", "l2", "D_cd", "D_kc", "D_ld", "D_lk",
                         "workspace"};
  for (int i = 0; i < 11; ++i)
    if ((rc = check_dev_ptr(ptrs[i], names[i]))) return rc;
  if (Yo && (rc = check_dev_ptr(Yo, "Yo"))) return rc;
  if (((uintptr_t)ws) & 255) return fail(CC3_E_INVAL, "workspace must be 256-byte aligned");
  DPlan p;
  make_dplan(no, nv, nchol, &p);
  if (ws_bytes < p.total)
    return fail(CC3_E_NOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, p.total);
  const bool acc = (flags & CC3_ACCUMULATE) != 0;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  double* Gw = (double*)(base + p.off_Gw);
  double* Gl = (double*)(base + p.off_Gl);
  double* Go = (double*)(base + p.off_Go);
  double* Go3 = (double*)(base + p.off_Go3);
  double* Jo = (double*)(base + p.off_Jo);
  double* F = (double*)(base + p.off_F);
  double* t2N = (double*)(base + p.off_t2N);
  double* l2M = (double*)(base + p.off_l2M);
  double* Y = (double*)(base + p.off_Y);
  double* Ppart = (double*)(base + p.off_part);
  double* Py = (double*)(base + p.off_py);
  double* Pkc = (double*)(base + p.off_pkc);
  int* dtri = (int*)(base + p.off_tri);
  int* dtask = (int*)(base + p.off_task);
  double* cubes = (double*)(base + p.off_cubes);
  // the Cholesky scratch, then the temporary (vv|ov) block, in the cube region
  const size_t o = no, v = nv, J = nchol;
  CholeskyScratch cs;
  {
    char* cr = base + p.off_cubes;
    size_t at = 0;
    auto take = [&](size_t bytes) { double* q = (double*)(cr + at); at = a256(at + bytes); return q; };
    cs.Lvv = take(J * v * v * 8);
    cs.Loo = take(J * o * o * 8);
    cs.LooT = take(J * o * o * 8);
    cs.LvoT = take(J * o * v * 8);
    cs.Lov = take(J * o * v * 8);
    cs.s = take(J * 8);
    cs.M = take(J * o * o * 8);
  }
  double* gtmp = (double*)(base + p.off_cubes + p.chol_bytes);
  const int64_t csl = (int64_t)p.cube, ss = (int64_t)no * csl;
  std::lock_guard<std::mutex> g(c->mu);
  Profiler* pf = &c->prof;
  HIPCHK(hipMemcpyAsync(dtri, p.htri.data(), p.htri.size() * sizeof(int), hipMemcpyHostToDevice,
                        st));
  if (p.ntask)
    HIPCHK(hipMemcpyAsync(dtask, p.htask.data(), p.htask.size() * sizeof(int),
                          hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // the host tables may go out of scope
  {
    Timer tm(pf, st, FAM_T1, 0.0, 0.0);
    launch_t1_transform(L, t1, cs, no, nv, nchol, st);
    launch_fock(t1, cs, F, no, nv, nchol, st);
  }
  {
    const double fl = 2.0 * J * (2.0 * v * v * v * o + o * o * v * v + 2.0 * o * o * o * v);
    Timer tm(pf, st, FAM_BUILD, fl, 0.0);
    launch_build_density_blocks(cs, Gw, Go, Jo, Go3, Gl, gtmp, no, nv, nchol, st);
  }
  launch_t2N(t2, t2N, no, nv, st);
  launch_d3_l2m(l2, l2M, no, nv, st);
  launch_fill(Y, (int64_t)o * o * o * v, 0.0, st);
  if (!acc) {
    launch_fill(D_cd, (int64_t)v * v, 0.0, st);
    launch_fill(D_kc, (int64_t)o * v, 0.0, st);
    launch_fill(D_ld, (int64_t)o * v, 0.0, st);
    launch_fill(D_lk, (int64_t)o * o, 0.0, st);
  }
  std::vector<int> kinds(no);
  for (int pr = 0; pr < p.npairs; ++pr) {
    const int i = p.pi[pr], j = p.pj[pr];
    const int* tb = dtri + (size_t)pr * no * 3;
    for (int k = 0; k < no; ++k) kinds[k] = tri_kind(i, j, k);
    const double wfl = wbuild_flops(no, nv, kinds.data(), no);
    {
      Timer tm(pf, st, FAM_W, wfl, 0.0);
      launch_wbuild_ex(0, t2, t2N, Gw, Go, tb, no, cubes, csl, ss, cube_pitch(nv), no, nv, false, st);
    }
    {
      Timer tm(pf, st, FAM_MIX, 0.0, 0.0);
      launch_mix3(false, eps, tb, no, cubes, ss, 0.0, l1, l2, Jo, F, no, nv, st);
    }
    {
      Timer tm(pf, st, FAM_L3, wfl, 0.0);
      launch_wbuild_ex(1, l2, l2M, Gl, Go3, tb, no, cubes, csl, ss, cube_pitch(nv), no, nv, false, st);
    }
    {
      Timer tm(pf, st, FAM_MIX, 0.0, 0.0);
      launch_mix3(true, eps, tb, no, cubes, ss, omega, l1, l2, Jo, F, no, nv, st);
    }
    const int nown = (i == j) ? j : j + 1;
    const int nt = p.ntasks[pr];
    const double dfl = (double)nown * 3 * 2.0 * v * v * v * v + (double)nt * 2.0 * v * v * v * (o + 1) +
                       2.0 * o * o * v * v * v;
    {
      Timer tm(pf, st, FAM_DENSITY, dfl, 0.0);
      launch_d3_cd(cubes, ss, tb, 0, nown, Ppart, D_cd, nv, st);
      launch_d3_vec(cubes, ss, dtask + (size_t)p.task0[pr] * D3_TASK_INTS, nt, t2, l2, Py, Pkc, Y,
                    D_kc, no, nv, st);
      launch_d3_gram(cubes, ss, 0, no, Ppart, D_lk, i > j ? -1.0 : -0.5, no, nv, st);
    }
    HIPCHK(hipGetLastError());
  }
  {
    Timer tm(pf, st, FAM_DENSITY, 2.0 * o * v * o * o * v, 0.0);
    launch_d3_ld(Y, t2, Ppart, D_ld, no, nv, st);
    if (Yo) launch_d3_yout(Y, Yo, no, nv, acc, st);
  }
  HIPCHK(hipGetLastError());
  return CC3_OK;
}
