// Contractions of the transition-density loop (Algorithm 3, the triples
// contributions to D^{m,0}) on gfx950, after the t3 and L3 builds and their mix.
//
// The loop runs over occupied pairs (i, j), i >= j: a batch holds the ordered
// triples (i, j, k) for every k, with t3 (tau), its contravariant form (tau~) and
// the contravariant left-state triples (L~) of each, cubes[slot][k][a][b][c].
//  - Triples (i, j, k) with k <= j are sorted, and each unordered triple is sorted
//    in exactly one pair: those ("owned") give, for each distinct ordering (p,q,r),
//      D_cd[c][d]   += 1/2 sum_ab L~_{pqr}[a,b,c] tau_{pqr}[a,b,d]
//      Y^o[c][l][p][r] += sum_ab L~_{pqr}[a,b,c] t2[l][q][a][b]
//      D_kc[r][c]   += sum_ab l2[p][q][a][b] tau~_{pqr}[a,b,c]
//    The six orderings pair up into three "mode" contractions, one per cube axis
//    holding the free index:  sum over orderings of the D_cd term
//    = w (G_0 + G_1 + G_2), G_m[c][d] = sum over the other two axes of L~ tau with
//    c, d on axis m, w = 1 for distinct indices and 1/2 with two equal.
//  - The occupied-occupied block, for which the paper runs a loop over virtual
//    triples, is  D_lk = -1/2 sum_{ij} sum_{abc} L~^{abc}_{ijk} tau^{abc}_{ijl}; per
//    pair it is the Gram matrix M_ij[k][l] = <L~_{ijk}, tau_{ijl}> of the batch's
//    cubes, and M_ji = M_ij (the simultaneous relabelling of (a,i) and (b,j)), so
//    D_lk -= 1/2 w_ij M_ij with w_ij = 2 for i > j, 1 for i == j.
// After the loop  D_ld = - sum_{cik} Y^o[c][l][i][k] t2[k][i][c][d].
// Every contraction goes to partial slabs reduced in a fixed order (no atomics).
#include "cc3_density.hpp"
#include "cc3_device.hpp"

namespace cc3 {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

typedef TileCfg<4, 2, 2, 4, 16> CdCfg;   // 128 x 128 (c, d) tiles
typedef TileCfg<8, 1, 1, 1, 16> VecCfg;  // 128 rows c x 16 columns (l, or the D_kc column)
typedef TileCfg<2, 2, 1, 1, 16> GrCfg;   // 32 x 32 tiles (Gram, D_ld)

// The six orderings of (i, j, k) in the order of itertools.permutations:
// ordering o takes the cube axes perm[o][0..2] for (a, b, c).
__constant__ int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// ---------------------------------------------------------------------------
// D_cd: mode contractions of the owned triples, split over the outer K axis
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CdCfg::NT) void k_d3_cd(const double* __restrict__ cubes, int64_t ss,
                                                     int z0, double* __restrict__ P, int nv,
                                                     int nch, int tiles_n) {
  typedef CdCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int m = blockIdx.y, t = blockIdx.z;
  const int ch = blockIdx.x % nch, tile = blockIdx.x / nch;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const int64_t nvl = nv, nv2 = nvl * nvl, rp = cube_pitch(nv), csl = cube_slot(nv);
  const int64_t S[3] = {nvl * rp, rp, 1};  // axis strides of the padded cubes
  const int u = (m == 0) ? 1 : 0, v = (m == 2) ? 1 : 2;  // the other two axes, u < v
  const double* Lc = cubes + D3_LC * ss + (int64_t)(z0 + t) * csl;
  const double* Ta = cubes + D3_TAU * ss + (int64_t)(z0 + t) * csl;
  const int u0 = (int)((int64_t)ch * nv / nch), u1 = (int)((int64_t)(ch + 1) * nv / nch);
  const int cs = (nv + T::BK - 1) / T::BK;
  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    const int uu = u0 + s / cs;
    k0 = (s % cs) * T::BK;
    A = make_opnd(Lc + uu * S[u], S[m], S[v], nv, nv, m == 2);
    B = make_opnd(Ta + uu * S[u], S[m], S[v], nv, nv, m == 2);
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>((u1 - u0) * cs, m0, n0, ops, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double* out = P + (((int64_t)t * 3 + m) * nch + ch) * nv2;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = m0 + acc_row<T>(wm, fm, lane, r), d = n0 + acc_col<T>(wn, fn, lane);
        if (c < nv && d < nv) out[(int64_t)c * nv + d] = acc[fm][fn][r];
      }
}

// D_cd[c][d] += sum over the owned triples (weight 1, or 1/2 with two equal
// indices), modes and chunks, in that order.
__global__ void k_d3_red_cd(const int* __restrict__ tri, int z0, int nown,
                            const double* __restrict__ P, double* __restrict__ D, int nv,
                            int nch) {
  const int64_t nv2 = (int64_t)nv * nv;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv2) return;
  double s = 0.0;
  for (int t = 0; t < nown; ++t) {
    const int i = tri[3 * (z0 + t)], j = tri[3 * (z0 + t) + 1], k = tri[3 * (z0 + t) + 2];
    const double w = (i != j && j != k && i != k) ? 1.0 : 0.5;
    double st = 0.0;
    for (int q = 0; q < 3 * nch; ++q) st += P[((int64_t)t * 3 * nch + q) * nv2 + e];
    s += w * st;
  }
  D[e] += s;
}

// ---------------------------------------------------------------------------
// Y^o and D_kc: per (owned triple, distinct ordering), rows c of the ordering's
// view, K = (a, b) split over a; the tasks (z, ordering, p, q, r) come from a
// table built on the host.
// ---------------------------------------------------------------------------
template <int KC>
__global__ __launch_bounds__(VecCfg::NT) void k_d3_vec(const double* __restrict__ cubes,
                                                       int64_t ss, const int* __restrict__ task,
                                                       const double* __restrict__ X,
                                                       double* __restrict__ P, int no, int nv,
                                                       int nch, int tiles_n) {
  typedef VecCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int ti = blockIdx.y;
  const int* tk = task + D3_TASK_INTS * ti;
  const int z = tk[0], ord = tk[1], p = tk[2], q = tk[3];
  const int ch = blockIdx.x % nch, tile = blockIdx.x / nch;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const int64_t nvl = nv, nv2 = nvl * nvl, rp = cube_pitch(nv), csl = cube_slot(nv);
  const int64_t S[3] = {nvl * rp, rp, 1};  // axis strides of the padded cubes
  const int axa = kPerm[ord][0], axb = kPerm[ord][1], axc = kPerm[ord][2];
  const double* U = cubes + (KC ? D3_TAUC : D3_LC) * ss + (int64_t)z * csl;
  // K = (a, b), split over its outer index.  When the view's a is the cube's contiguous
  // axis, K runs in (b, a) order instead, so that the A loads run along a; B then reads
  // the pair-symmetric copy of its row, t2[l][q][a][b] = t2[q][l][b][a] and
  // l2[p][q][a][b] = l2[q][p][b][a], with a contiguous as well.
  const bool ba = (axa == 2);
  const int a0 = (int)((int64_t)ch * nv / nch), a1 = (int)((int64_t)(ch + 1) * nv / nch);
  const int cs = (nv + T::BK - 1) / T::BK;
  const int ncol = KC ? 1 : no;
  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    const int oo = a0 + s / cs;  // a, or b when ba
    k0 = (s % cs) * T::BK;
    if (!ba) {
      A = make_opnd(U + oo * S[axa], S[axc], S[axb], nv, nv, S[axc] == 1);
      if (KC)  // the single row l2[p][q][a][.]
        B = make_opnd(X + ((int64_t)p * no + q) * nv2 + (int64_t)oo * nv, 0, 1, 1, nv, false);
      else  // rows l of t2[l][q][a][.]
        B = make_opnd(X + (int64_t)q * nv2 + (int64_t)oo * nv, (int64_t)no * nv2, 1, no, nv, false);
    } else {
      A = make_opnd(U + oo * S[axb], S[axc], S[axa], nv, nv, false);
      if (KC)  // l2[q][p][b][.]
        B = make_opnd(X + ((int64_t)q * no + p) * nv2 + (int64_t)oo * nv, 0, 1, 1, nv, false);
      else  // rows l of t2[q][l][b][.]
        B = make_opnd(X + (int64_t)q * no * nv2 + (int64_t)oo * nv, nv2, 1, no, nv, false);
    }
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>((a1 - a0) * cs, m0, n0, ops, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double* out = P + ((int64_t)ti * nch + ch) * nvl * ncol;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = m0 + acc_row<T>(wm, fm, lane, r), l = n0 + acc_col<T>(wn, fn, lane);
        if (c < nv && l < ncol) out[(int64_t)c * ncol + l] = acc[fm][fn][r];
      }
}

// Y'[l][r][p][c] (= Y^o[c][l][p][r]) += the chunk sums of the tasks with that (p, r),
// in task order; one block of (l, c) per (p, r).
__global__ void k_d3_red_y(const int* __restrict__ task, int ntask, const double* __restrict__ P,
                           double* __restrict__ Y, int no, int nv, int nch) {
  const int p = blockIdx.y / no, r = blockIdx.y % no;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // c * no + l
  if (e >= (int64_t)nv * no) return;
  const int c = (int)(e / no), l = (int)(e % no);
  const int64_t slab = (int64_t)nv * no;
  double s = 0.0;
  bool any = false;
  for (int t = 0; t < ntask; ++t) {
    const int* tk = task + D3_TASK_INTS * t;
    if (tk[2] != p || tk[4] != r) continue;
    any = true;
    for (int ch = 0; ch < nch; ++ch) s += P[((int64_t)t * nch + ch) * slab + e];
  }
  if (any) Y[(((int64_t)l * no + r) * no + p) * nv + c] += s;
}

// D_kc[r][c] += the chunk sums of the tasks with that r, in task order.
__global__ void k_d3_red_kc(const int* __restrict__ task, int ntask, const double* __restrict__ P,
                            double* __restrict__ D, int no, int nv, int nch) {
  const int r = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nv) return;
  double s = 0.0;
  for (int t = 0; t < ntask; ++t) {
    if (task[D3_TASK_INTS * t + 4] != r) continue;
    for (int ch = 0; ch < nch; ++ch) s += P[((int64_t)t * nch + ch) * nv + c];
  }
  D[(int64_t)r * nv + c] += s;
}

// ---------------------------------------------------------------------------
// Gram matrix of a pair: M[k][l] = <L~_k, tau_l> over the whole cube, split over K
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(GrCfg::NT) void k_d3_gram(const double* __restrict__ cubes,
                                                       int64_t ss, int z0, int nz,
                                                       double* __restrict__ P, int nv, int nch,
                                                       int tiles_n) {
  typedef GrCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int ch = blockIdx.x % nch, tile = blockIdx.x / nch;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  // K = the whole padded cube; its padding columns hold zeros in both operands
  const int64_t cs = cube_slot(nv);
  const int K = (int)cs;
  const int S = (K + T::BK - 1) / T::BK;
  const int s0 = (int)((int64_t)ch * S / nch), s1 = (int)((int64_t)(ch + 1) * S / nch);
  const double* Lc = cubes + D3_LC * ss + (int64_t)z0 * cs;
  const double* Ta = cubes + D3_TAU * ss + (int64_t)z0 * cs;
  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    k0 = (s0 + s) * T::BK;
    A = make_opnd(Lc, cs, 1, nz, K, false);
    B = make_opnd(Ta, cs, 1, nz, K, false);
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>(s1 - s0, m0, n0, ops, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double* out = P + (int64_t)ch * nz * nz;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = m0 + acc_row<T>(wm, fm, lane, r), l = n0 + acc_col<T>(wn, fn, lane);
        if (k < nz && l < nz) out[(int64_t)k * nz + l] = acc[fm][fn][r];
      }
}

// D_lk[l][k] += scale * sum over chunks of M[k][l]
// One workgroup per element D_lk[l][k]: thread t sums the chunks t, t + 256, ... in
// order, then a fixed binary tree over the 256 partial sums (deterministic).
__global__ __launch_bounds__(256) void k_d3_red_lk(const double* __restrict__ P,
                                                   double* __restrict__ D, int no, int nch,
                                                   double scale) {
  __shared__ double part[256];
  const int e = blockIdx.x;
  const int l = e / no, k = e % no;
  double s = 0.0;
  for (int ch = threadIdx.x; ch < nch; ch += 256) s += P[(int64_t)ch * no * no + (int64_t)k * no + l];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) D[e] += scale * part[0];
}

// ---------------------------------------------------------------------------
// D_ld = - sum_{k,i,c} Y'[l][k][i][c] t2[k][i][c][d]: rows l, columns d, K = (k,i,c)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(GrCfg::NT) void k_d3_ld(const double* __restrict__ Y,
                                                     const double* __restrict__ t2,
                                                     double* __restrict__ P, int no, int nv,
                                                     int nch, int tiles_n) {
  typedef GrCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int ch = blockIdx.x % nch, tile = blockIdx.x / nch;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const int K = no * no * nv;
  const int S = (K + T::BK - 1) / T::BK;
  const int s0 = (int)((int64_t)ch * S / nch), s1 = (int)((int64_t)(ch + 1) * S / nch);
  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    k0 = (s0 + s) * T::BK;
    A = make_opnd(Y, K, 1, no, K, false);
    B = make_opnd(t2, 1, nv, nv, K, true);
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>(s1 - s0, m0, n0, ops, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double* out = P + (int64_t)ch * no * nv;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int l = m0 + acc_row<T>(wm, fm, lane, r), d = n0 + acc_col<T>(wn, fn, lane);
        if (l < no && d < nv) out[(int64_t)l * nv + d] = acc[fm][fn][r];
      }
}

__global__ void k_d3_red_ld(const double* __restrict__ P, double* __restrict__ D, int no, int nv,
                            int nch) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)no * nv) return;
  double s = 0.0;
  for (int ch = 0; ch < nch; ++ch) s += P[(int64_t)ch * no * nv + e];
  D[e] -= s;
}

// Y^o[c][l][i][k] (+)= Y'[l][k][i][c]
__global__ void k_d3_yout(const double* __restrict__ Y, double* __restrict__ Yo, int no, int nv,
                          int accumulate) {
  const int64_t n = (int64_t)nv * no * no * no;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int k = (int)(e % no), i = (int)((e / no) % no), l = (int)((e / (no * no)) % no);
  const int c = (int)(e / ((int64_t)no * no * no));
  const double v = Y[(((int64_t)l * no + k) * no + i) * nv + c];
  Yo[e] = accumulate ? Yo[e] + v : v;
}

// l2M[r][y][x][l] = -l2[l][r][x][y]
__global__ void k_d3_l2m(const double* __restrict__ l2, double* __restrict__ l2M, int no, int nv) {
  const int64_t nvl = nv, n = (int64_t)no * no * nvl * nvl;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int l = (int)(e % no), x = (int)((e / no) % nvl), y = (int)((e / (no * nvl)) % nvl);
  const int r = (int)(e / (no * nvl * nvl));
  l2M[e] = -l2[(((int64_t)l * no + r) * nvl + x) * nvl + y];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int d3_cd_chunks(int nv, int nown) {
  const int t = (nv + CdCfg::BM - 1) / CdCfg::BM;
  int n = (2048 + 3 * t * t * nown - 1) / (3 * t * t * (nown > 0 ? nown : 1));
  return n < 1 ? 1 : (n > nv ? nv : n);
}

int d3_vec_chunks(int nv, int ntask, int ncol) {
  const int t = ((nv + VecCfg::BM - 1) / VecCfg::BM) * ((ncol + VecCfg::BN - 1) / VecCfg::BN);
  int n = (2048 + t * ntask - 1) / (t * (ntask > 0 ? ntask : 1));
  return n < 1 ? 1 : (n > nv ? nv : n);
}

int d3_gram_chunks(int nv, int nz) {
  const int t = (nz + GrCfg::BM - 1) / GrCfg::BM;
  const int S = (int)((cube_slot(nv) + GrCfg::BK - 1) / GrCfg::BK);
  int n = (2048 + t * t - 1) / (t * t);
  return n > S ? S : n;
}

int d3_ld_chunks(int no, int nv) {
  const int t = ((no + GrCfg::BM - 1) / GrCfg::BM) * ((nv + GrCfg::BN - 1) / GrCfg::BN);
  const int S = (no * no * nv + GrCfg::BK - 1) / GrCfg::BK;
  int n = (1024 + t - 1) / t;
  return n > S ? S : n;
}

void launch_d3_cd(const double* cubes, int64_t ss, const int* tri, int z0, int nown, double* P,
                  double* Dcd, int nv, hipStream_t st) {
  if (nown <= 0) return;
  typedef CdCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + T::BN - 1) / T::BN;
  const int nch = d3_cd_chunks(nv, nown);
  hipLaunchKernelGGL(k_d3_cd, dim3(tm * tn * nch, 3, nown), dim3(T::NT), 0, st, cubes, ss, z0, P,
                     nv, nch, tn);
  hipLaunchKernelGGL(k_d3_red_cd, dim3(nblk((int64_t)nv * nv, 256)), dim3(256), 0, st, tri, z0,
                     nown, P, Dcd, nv, nch);
}

void launch_d3_vec(const double* cubes, int64_t ss, const int* task, int ntask, const double* t2,
                   const double* l2, double* Py, double* Pkc, double* Y, double* Dkc, int no,
                   int nv, hipStream_t st) {
  if (ntask <= 0) return;
  typedef VecCfg T;
  const int tm = (nv + T::BM - 1) / T::BM;
  {
    const int tn = (no + T::BN - 1) / T::BN, nch = d3_vec_chunks(nv, ntask, no);
    hipLaunchKernelGGL(k_d3_vec<0>, dim3(tm * tn * nch, ntask), dim3(T::NT), 0, st, cubes, ss,
                       task, t2, Py, no, nv, nch, tn);
    hipLaunchKernelGGL(k_d3_red_y, dim3(nblk((int64_t)nv * no, 256), no * no), dim3(256), 0, st,
                       task, ntask, Py, Y, no, nv, nch);
  }
  {
    const int nch = d3_vec_chunks(nv, ntask, 1);
    hipLaunchKernelGGL(k_d3_vec<1>, dim3(tm * nch, ntask), dim3(T::NT), 0, st, cubes, ss, task, l2,
                       Pkc, no, nv, nch, 1);
    hipLaunchKernelGGL(k_d3_red_kc, dim3(nblk(nv, 256), no), dim3(256), 0, st, task, ntask, Pkc,
                       Dkc, no, nv, nch);
  }
}

void launch_d3_gram(const double* cubes, int64_t ss, int z0, int nz, double* P, double* Dlk,
                    double scale, int no, int nv, hipStream_t st) {
  typedef GrCfg T;
  const int t = (nz + T::BM - 1) / T::BM;
  const int nch = d3_gram_chunks(nv, nz);
  hipLaunchKernelGGL(k_d3_gram, dim3(t * t * nch), dim3(T::NT), 0, st, cubes, ss, z0, nz, P, nv,
                     nch, t);
  hipLaunchKernelGGL(k_d3_red_lk, dim3(no * no), dim3(256), 0, st, P, Dlk, no, nch, scale);
}

void launch_d3_ld(const double* Y, const double* t2, double* P, double* Dld, int no, int nv,
                  hipStream_t st) {
  typedef GrCfg T;
  const int tm = (no + T::BM - 1) / T::BM, tn = (nv + T::BN - 1) / T::BN;
  const int nch = d3_ld_chunks(no, nv);
  hipLaunchKernelGGL(k_d3_ld, dim3(tm * tn * nch), dim3(T::NT), 0, st, Y, t2, P, no, nv, nch, tn);
  hipLaunchKernelGGL(k_d3_red_ld, dim3(nblk((int64_t)no * nv, 256)), dim3(256), 0, st, P, Dld, no,
                     nv, nch);
}

void launch_d3_yout(const double* Y, double* Yo, int no, int nv, bool accumulate, hipStream_t st) {
  const int64_t n = (int64_t)nv * no * no * no;
  hipLaunchKernelGGL(k_d3_yout, dim3(nblk(n, 256)), dim3(256), 0, st, Y, Yo, no, nv,
                     accumulate ? 1 : 0);
}

void launch_d3_l2m(const double* l2, double* l2M, int no, int nv, hipStream_t st) {
  const int64_t n = (int64_t)no * no * nv * nv;
  hipLaunchKernelGGL(k_d3_l2m, dim3(nblk(n, 256)), dim3(256), 0, st, l2, l2M, no, nv);
}

size_t d3_partial_doubles(int no, int nv) {
  // the largest partial-slab need of any launch of the loop
  size_t cd = 0, vy = 0, vk = 0;
  for (int nown = 1; nown <= no; ++nown)
    cd = std::max(cd, (size_t)nown * 3 * d3_cd_chunks(nv, nown) * nv * nv);
  for (int nt = 1; nt <= 6 * no; ++nt) {
    vy = std::max(vy, (size_t)nt * d3_vec_chunks(nv, nt, no) * nv * no);
    vk = std::max(vk, (size_t)nt * d3_vec_chunks(nv, nt, 1) * nv);
  }
  const size_t gr = (size_t)d3_gram_chunks(nv, no) * no * no;
  const size_t ld = (size_t)d3_ld_chunks(no, nv) * no * nv;
  // D_cd, Gram and D_ld partials share one region; Y^o and D_kc have their own
  return std::max(std::max(cd, gr), ld) + vy + vk;
}

}  // namespace cc3
