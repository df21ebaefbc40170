// The triple loop of Algorithm 1 (CC3 ground-state equations) on gfx950.
//
// For a batch of unordered occupied triples i >= j >= k (not all equal):
//
//  k_wbuild  (FP64 MFMA)  the six terms B_pqr[x,y,z] = sum_d t2[p][q][x][d] g_{ydzr}
//            - sum_l t2[p][l][x][y] g_{lqzr} of the permutation operator, paired
//            two per "plane" so that each workgroup writes one nv x nv plane:
//              P0[b][a][c] = B_ijk[a,b,c] + B_kji[c,b,a]
//              P1[a][b][c] = B_jik[b,a,c] + B_kij[c,a,b]
//              P2[c][a][b] = B_ikj[a,c,b] + B_jki[b,c,a]
//            so that X = P B = P0[b][a][c] + P1[a][b][c] + P2[c][a][b].  With two
//            equal occupied indices three of the six terms repeat and are not
//            recomputed.
//  k_mix     (LDS)  per S3-orbit of 8x8x8 virtual blocks: X, the denominator
//            division tau = -X / eps^{abc}_{ijk}, and the contravariant
//            tau~ = 4 tau^{abc} - 2 tau^{acb} - 2 tau^{cba} - 2 tau^{bac} + tau^{bca} + tau^{cab},
//            written as tau~[a][b][c] and its transpose tau~T[a][c][b].
//  k_omega   (FP64 MFMA)  for each distinct occupied permutation (p,q,r), with
//            U = tau~_{pqr} read from tau~ or tau~T, one GEMM over K = (b, c):
//              Ot2[p][q][a][d] += sum_bc U[a,b,c] g_{dbrc}    (columns d < nv)
//              Ot1[p][a]       += sum_bc U[a,b,c] g_{qbrc}    (column nv)
//              Ot2[p][l][a][b] += sum_c  U[a,b,c] (delta_lq F_rc - g_{qlrc})  (separate
//                                 accumulator blocks, flushed after every b)
#include "cc3_device.hpp"
#include "cc3_internal.hpp"

namespace cc3 {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// triple kinds
enum { TRI_DISTINCT = 0, TRI_IJ = 1, TRI_JK = 2 };

__device__ inline int tri_kind(int i, int j, int k) {
  if (i == j) return TRI_IJ;  // i == j > k
  if (j == k) return TRI_JK;  // i > j == k
  return TRI_DISTINCT;
}

// cube slots of one triple's workspace
enum { SLOT_P0 = 0, SLOT_P1 = 1, SLOT_P2 = 2, SLOT_TT = 3, SLOT_TTT = 4, NSLOT = 5 };

// ---------------------------------------------------------------------------
// W build
// ---------------------------------------------------------------------------
typedef TileCfg<4, 1, 2, 8> WCfg;  // 128 x 128 output plane tile

__global__ __launch_bounds__(WCfg::NT) void k_wbuild(const double* __restrict__ t2,
                                                     const double* __restrict__ Gw,
                                                     const double* __restrict__ Go,
                                                     const int* __restrict__ tri,
                                                     double* __restrict__ cubes, int no, int nv,
                                                     int tiles_m, int tiles_n, int all_terms) {
  typedef WCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int tpp = tiles_m * tiles_n;
  const int y = blockIdx.x / tpp;
  const int tile = blockIdx.x % tpp;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const int plane = blockIdx.y;
  const int z = blockIdx.z;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  const int kind = all_terms ? TRI_DISTINCT : tri_kind(i, j, k);
  // plane 1 repeats plane 0 when i == j, plane 2 repeats plane 0 when j == k
  if ((kind == TRI_IJ && plane == 1) || (kind == TRI_JK && plane == 2)) return;
  const bool two = (kind == TRI_DISTINCT) || plane == 0;
  int p1, q1, r1, p2, q2, r2;
  if (plane == 0) { p1 = i; q1 = j; r1 = k; p2 = k; q2 = j; r2 = i; }
  else if (plane == 1) { p1 = j; q1 = i; r1 = k; p2 = k; q2 = i; r2 = j; }
  else { p1 = i; q1 = k; r1 = j; p2 = j; q2 = k; r2 = i; }

  const int64_t nv2 = (int64_t)nv * nv, nv3 = nv2 * nv;
  const int nvs = (nv + T::BK - 1) / T::BK, nos = (no + T::BK - 1) / T::BK;
  const int nsteps = two ? 2 * (nvs + nos) : (nvs + nos);

  // term 1: Acc[m][n] += sum_d t2[p1][q1][m][d] Gw[r1][y][d][n] - sum_l t2[p1][l][m][y] Go[q1][r1][l][n]
  // term 2: Acc[m][n] += sum_d Gw[r2][y][d][m] t2[p2][q2][n][d] - sum_l Go[q2][r2][l][m] t2[p2][l][n][y]
  const double* a0 = t2 + ((int64_t)p1 * no + q1) * nv2;
  const double* b0 = Gw + ((int64_t)r1 * nv + y) * nv2;
  const double* a1 = t2 + (int64_t)p1 * no * nv2 + y;
  const double* b1 = Go + ((int64_t)q1 * no + r1) * no * nv;
  const double* a2 = Gw + ((int64_t)r2 * nv + y) * nv2;
  const double* b2 = t2 + ((int64_t)p2 * no + q2) * nv2;
  const double* a3 = Go + ((int64_t)q2 * no + r2) * no * nv;
  const double* b3 = t2 + (int64_t)p2 * no * nv2 + y;

  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    int seg = 0, ls = s;
    if (ls >= nvs) { ls -= nvs; seg = 1;
      if (ls >= nos) { ls -= nos; seg = 2;
        if (ls >= nvs) { ls -= nvs; seg = 3; } } }
    k0 = ls * T::BK;
    if (seg == 0) {
      A = make_opnd(a0, nv, 1, nv, nv, 1.0, false);
      B = make_opnd(b0, 1, nv, nv, nv, 1.0, true);
    } else if (seg == 1) {
      A = make_opnd(a1, nv, nv2, nv, no, -1.0, true);
      B = make_opnd(b1, 1, nv, nv, no, 1.0, true);
    } else if (seg == 2) {
      A = make_opnd(a2, 1, nv, nv, nv, 1.0, true);
      B = make_opnd(b2, nv, 1, nv, nv, 1.0, false);
    } else {
      A = make_opnd(a3, 1, nv, nv, no, 1.0, true);
      B = make_opnd(b3, nv, nv2, nv, no, -1.0, true);
    }
  };
  auto none = [](int) {};
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>(nsteps, m0, n0, ops, none, acc, lds);

  double* out = cubes + ((int64_t)z * NSLOT + plane) * nv3 + (int64_t)y * nv2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + acc_row<T>(wm, fm, lane, r);
        const int n = n0 + acc_col<T>(wn, fn, lane);
        if (m < nv && n < nv) out[(int64_t)m * nv + n] = acc[fm][fn][r];
      }
}

void launch_wbuild(const double* t2, const Blocks& b, const int* tri, int ntri, double* cubes,
                   int no, int nv, bool all_terms, hipStream_t st) {
  typedef WCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + T::BN - 1) / T::BN;
  hipLaunchKernelGGL(k_wbuild, dim3(nv * tm * tn, 3, ntri), dim3(T::NT), 0, st, t2, b.Gw, b.Go,
                     tri, cubes, no, nv, tm, tn, all_terms ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Mix: X, tau, tau~ on the S3 orbit of an 8x8x8 block triple (A <= B <= C).
// ---------------------------------------------------------------------------
#define MT 8
#define MT3 (MT * MT * MT)

// the six orientations of a block triple, as positions into (A, B, C)
__constant__ int c_orient[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__device__ inline int orient_of(int p0, int p1) {
  // the orientation index whose first two positions are (p0, p1)
  return p0 == 0 ? (p1 == 1 ? 0 : 1) : (p0 == 1 ? (p1 == 0 ? 2 : 3) : (p1 == 0 ? 4 : 5));
}

__device__ inline void decode_block_triple(int idx, int& A, int& B, int& C) {
  // lexicographic (C, B, A) with A <= B <= C
  int c = 0;
  while ((c + 1) * (c + 2) * (c + 3) / 6 <= idx) ++c;
  idx -= c * (c + 1) * (c + 2) / 6;
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= idx) ++b;
  idx -= b * (b + 1) / 2;
  A = idx; B = b; C = c;
}

__device__ inline double xval(const double* __restrict__ cz, int kind, int64_t nv, int a, int b,
                              int c) {
  const int64_t nv2 = nv * nv, nv3 = nv2 * nv;
  const double* P0 = cz + SLOT_P0 * nv3;
  const double* P1 = cz + SLOT_P1 * nv3;
  const double* P2 = cz + SLOT_P2 * nv3;
  if (kind == TRI_DISTINCT)
    return P0[b * nv2 + a * nv + c] + P1[a * nv2 + b * nv + c] + P2[c * nv2 + a * nv + b];
  if (kind == TRI_IJ)  // P1 = P0, P2[c][a][b] = Q[c][a][b] + Q[c][b][a]
    return P0[b * nv2 + a * nv + c] + P0[a * nv2 + b * nv + c] + P2[c * nv2 + a * nv + b] +
           P2[c * nv2 + b * nv + a];
  // TRI_JK: P2 = P0, P1[a][b][c] = R[a][b][c] + R[a][c][b]
  return P0[b * nv2 + a * nv + c] + P1[a * nv2 + b * nv + c] + P1[a * nv2 + c * nv + b] +
         P0[c * nv2 + a * nv + b];
}

__global__ __launch_bounds__(256) void k_mix(const double* __restrict__ eps,
                                             const int* __restrict__ tri,
                                             double* __restrict__ cubes, int no, int nv) {
  __shared__ double Xs[6 * MT3];
  __shared__ double Ts[6 * MT3];
  __shared__ int blk3[3];
  const int z = blockIdx.y;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  const int kind = tri_kind(i, j, k);
  const int64_t nvl = nv, nv3 = nvl * nvl * nvl;
  double* cz = cubes + (int64_t)z * NSLOT * nv3;
  if (threadIdx.x == 0) {
    int A, B, C;
    decode_block_triple(blockIdx.x, A, B, C);
    blk3[0] = A; blk3[1] = B; blk3[2] = C;
  }
  __syncthreads();
  const double eijk = eps[i] + eps[j] + eps[k];
  // 1. X on the orbit
  for (int e = threadIdx.x; e < 6 * MT3; e += 256) {
    const int o = e / MT3, u = (e / (MT * MT)) % MT, v = (e / MT) % MT, w = e % MT;
    const int a = blk3[c_orient[o][0]] * MT + u;
    const int b = blk3[c_orient[o][1]] * MT + v;
    const int c = blk3[c_orient[o][2]] * MT + w;
    Xs[e] = (a < nv && b < nv && c < nv) ? xval(cz, kind, nvl, a, b, c) : 0.0;
  }
  __syncthreads();
  // 2. tau~ on the orbit
  for (int e = threadIdx.x; e < 6 * MT3; e += 256) {
    const int o = e / MT3, u = (e / (MT * MT)) % MT, v = (e / MT) % MT, w = e % MT;
    const int p0 = c_orient[o][0], p1 = c_orient[o][1], p2 = c_orient[o][2];
    const int a = blk3[p0] * MT + u, b = blk3[p1] * MT + v, c = blk3[p2] * MT + w;
    double t = 0.0;
    if (a < nv && b < nv && c < nv) {
      // X at permuted virtual labels: (a,c,b), (c,b,a), (b,a,c), (b,c,a), (c,a,b)
      const double x_abc = Xs[e];
      const double x_acb = Xs[orient_of(p0, p2) * MT3 + (u * MT + w) * MT + v];
      const double x_cba = Xs[orient_of(p2, p1) * MT3 + (w * MT + v) * MT + u];
      const double x_bac = Xs[orient_of(p1, p0) * MT3 + (v * MT + u) * MT + w];
      const double x_bca = Xs[orient_of(p1, p2) * MT3 + (v * MT + w) * MT + u];
      const double x_cab = Xs[orient_of(p2, p0) * MT3 + (w * MT + u) * MT + v];
      const double D = eps[no + a] + eps[no + b] + eps[no + c] - eijk;
      t = -(4.0 * x_abc - 2.0 * x_acb - 2.0 * x_cba - 2.0 * x_bac + x_bca + x_cab) / D;
    }
    Ts[e] = t;
  }
  __syncthreads();
  // 3. write tau~[a][b][c] (w fastest) and tau~T[a][c][b] (v fastest), skipping
  //    orientations that repeat an earlier one (equal blocks)
  double* TT = cz + SLOT_TT * nv3;
  double* TTT = cz + SLOT_TTT * nv3;
  for (int e = threadIdx.x; e < 6 * MT3; e += 256) {
    const int o = e / MT3;
    bool dup = false;
    for (int o2 = 0; o2 < o; ++o2)
      dup |= (blk3[c_orient[o2][0]] == blk3[c_orient[o][0]] &&
              blk3[c_orient[o2][1]] == blk3[c_orient[o][1]] &&
              blk3[c_orient[o2][2]] == blk3[c_orient[o][2]]);
    if (dup) continue;
    {  // tau~, element (u, v, w) with w fastest
      const int u = (e / (MT * MT)) % MT, v = (e / MT) % MT, w = e % MT;
      const int a = blk3[c_orient[o][0]] * MT + u, b = blk3[c_orient[o][1]] * MT + v,
                c = blk3[c_orient[o][2]] * MT + w;
      if (a < nv && b < nv && c < nv) TT[(a * nvl + b) * nvl + c] = Ts[e];
    }
    {  // tau~T, element (u, w, v) with v fastest
      const int u = (e / (MT * MT)) % MT, w = (e / MT) % MT, v = e % MT;
      const int a = blk3[c_orient[o][0]] * MT + u, b = blk3[c_orient[o][1]] * MT + v,
                c = blk3[c_orient[o][2]] * MT + w;
      if (a < nv && b < nv && c < nv)
        TTT[(a * nvl + c) * nvl + b] = Ts[o * MT3 + (u * MT + v) * MT + w];
    }
  }
}

void launch_mix(const double* eps, const int* tri, int ntri, double* cubes, int no, int nv,
                hipStream_t st) {
  const int nb = (nv + MT - 1) / MT;
  const int nbt = nb * (nb + 1) * (nb + 2) / 6;
  hipLaunchKernelGGL(k_mix, dim3(nbt, ntri), dim3(256), 0, st, eps, tri, cubes, no, nv);
}

// tau^{abc}_{ijk} = -X / eps^{abc}_{ijk} for one ordered triple whose six terms were all built
__global__ void k_tau_export(const double* __restrict__ eps, const int* __restrict__ tri,
                             const double* __restrict__ cubes, double* __restrict__ tau, int no,
                             int nv) {
  const int64_t nvl = nv, nv3 = nvl * nvl * nvl;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv3) return;
  const int a = (int)(e / (nvl * nvl)), b = (int)((e / nvl) % nvl), c = (int)(e % nvl);
  const int i = tri[0], j = tri[1], k = tri[2];
  const double X = xval(cubes, TRI_DISTINCT, nvl, a, b, c);
  tau[e] = -X / (eps[no + a] + eps[no + b] + eps[no + c] - eps[i] - eps[j] - eps[k]);
}

void launch_tau_export(const double* eps, const int* tri, const double* cubes, double* tau, int no,
                       int nv, hipStream_t st) {
  const int64_t nv3 = (int64_t)nv * nv * nv;
  hipLaunchKernelGGL(k_tau_export, dim3(nblk(nv3, 256)), dim3(256), 0, st, eps, tri, cubes, tau,
                     no, nv);
}

// ---------------------------------------------------------------------------
// Omega contraction
// ---------------------------------------------------------------------------
// Output columns of one (triple, permutation) GEMM over K = (b, c):
//   n < nv       : d of Ot2[p][q][a][d]    (B = Gv[r][b][d][c])
//   n == nv      : Ot1[p][a]               (B = Jo[q][r][b][c])
// plus, in separate accumulator blocks owned by the first N tile,
//   l < no       : Ot2[p][l][a][b]         (B = Hs[q][r][l][c]), flushed per b.
typedef TileCfg<4, 1, 2, 8> OCfg;  // 128 x 128 for the (d, Omega1) columns

template <int FNO>
__global__ __launch_bounds__(OCfg::NT) void k_omega(
    const double* __restrict__ cubes, const double* __restrict__ Gv, const double* __restrict__ Jo,
    const double* __restrict__ Hs, const int* __restrict__ tri, double* __restrict__ Ot1,
    double* __restrict__ Ot2, int no, int nv, int bchunk, int nbchunks, int tiles_n) {
  typedef OCfg T;
  constexpr int BO = 16 * FNO;            // oo columns per tile
  constexpr int LDO = BO + 16;
  constexpr int EO = (BO * T::BK + T::NT - 1) / T::NT;
  constexpr int STAGE = T::BK * (T::LDA + T::LDB + LDO);
  __shared__ double lds[2 * STAGE];
  const int pi = blockIdx.y;
  const int z = blockIdx.z;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  const int kind = tri_kind(i, j, k);
  // distinct occupied permutations: all six, {0,2,3} when i == j, {0,1,2} when j == k
  if (kind == TRI_IJ && (pi == 1 || pi == 4 || pi == 5)) return;
  if (kind == TRI_JK && pi >= 3) return;
  int p, q, r;
  switch (pi) {
    case 0: p = i; q = j; r = k; break;
    case 1: p = j; q = i; r = k; break;
    case 2: p = k; q = j; r = i; break;
    case 3: p = i; q = k; r = j; break;
    case 4: p = j; q = k; r = i; break;
    default: p = k; q = i; r = j; break;
  }
  const int bc = blockIdx.x % nbchunks;
  const int tile = blockIdx.x / nbchunks;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const bool do_oo = (tile % tiles_n) == 0;
  const int bb0 = bc * bchunk;
  const int bb1 = min(nv, bb0 + bchunk);
  if (bb0 >= bb1) return;

  const int64_t nvl = nv, nv2 = nvl * nvl, nv3 = nv2 * nvl;
  const double* TT = cubes + ((int64_t)z * NSLOT + SLOT_TT) * nv3;
  const double* TTT = cubes + ((int64_t)z * NSLOT + SLOT_TTT) * nv3;
  // U_pi[a, b, c] at fixed b as a strided (a, c) view: base + b * sbb, (sm, sk)
  const double* ub;
  int64_t sbb, sm, sk;
  switch (pi) {
    case 0: ub = TT; sbb = nvl; sm = nv2; sk = 1; break;     // tau~[a][b][c]
    case 1: ub = TT; sbb = nv2; sm = nvl; sk = 1; break;     // tau~[b][a][c]
    case 2: ub = TT; sbb = nvl; sm = 1; sk = nv2; break;     // tau~[c][b][a]
    case 3: ub = TTT; sbb = nvl; sm = nv2; sk = 1; break;    // tau~[a][c][b] = tau~T[a][b][c]
    case 4: ub = TTT; sbb = nvl; sm = 1; sk = nv2; break;    // tau~[c][a][b] = tau~T[c][b][a]
    default: ub = TT; sbb = nv2; sm = 1; sk = nvl; break;    // tau~[b][c][a]
  }
  const bool afast = (sm == 1);
  const int cs = (nv + T::BK - 1) / T::BK;  // c steps per b
  const int nsteps = (bb1 - bb0) * cs;
  const double* Gr = Gv + (int64_t)r * nv3;
  const double* Jqr = Jo + ((int64_t)q * no + r) * nv2;
  const double* Hqr = Hs + ((int64_t)q * no + r) * no * nvl;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  d4v acc[T::FM][T::FN];
  d4v aco[T::FM][FNO];
  zero_acc<T>(acc);
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int f = 0; f < FNO; ++f) aco[fm][f] = d4v{0.0, 0.0, 0.0, 0.0};
  double ra[T::EA], rb[T::EB], ro[EO];

  auto load = [&](int s) {
    const int b = bb0 + s / cs, c0 = (s % cs) * T::BK;
    const Opnd A = make_opnd(ub + (int64_t)b * sbb, sm, sk, nv, nv, 1.0, afast);
    load_stage<T::BM, T::BK, T::EA, T::NT>(A, m0, c0, ra, tid);
    const double* gb = Gr + (int64_t)b * nv2;
    const double* jb = Jqr + (int64_t)b * nvl;
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int idx = e * T::NT + tid;
      const int kk = idx % T::BK, n = n0 + idx / T::BK, c = c0 + kk;
      double v = 0.0;
      if (idx < T::BN * T::BK && c < nv) {
        if (n < nv) v = gb[(int64_t)n * nvl + c];
        else if (n == nv) v = jb[c];
      }
      rb[e] = v;
    }
    if (do_oo) {
#pragma unroll
      for (int e = 0; e < EO; ++e) {
        const int idx = e * T::NT + tid;
        const int kk = idx % T::BK, l = idx / T::BK, c = c0 + kk;
        ro[e] = (idx < BO * T::BK && c < nv && l < no) ? Hqr[(int64_t)l * nvl + c] : 0.0;
      }
    }
  };
  auto store = [&](double* st) {
    store_stage<T::BM, T::BK, T::EA, T::NT, T::LDA>(afast, ra, st, tid);
    store_stage<T::BN, T::BK, T::EB, T::NT, T::LDB>(false, rb, st + T::BK * T::LDA, tid);
    if (do_oo) store_stage<BO, T::BK, EO, T::NT, LDO>(false, ro, st + T::BK * (T::LDA + T::LDB), tid);
  };

  load(0);
  store(lds);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    double* cur = lds + (s & 1) * STAGE;
    double* nxt = lds + ((s + 1) & 1) * STAGE;
    const bool more = (s + 1 < nsteps);
    if (more) load(s + 1);
    mfma_stage<T>(cur, cur + T::BK * T::LDA, acc, lane, wm, wn);
    if (do_oo) {
      const double* so = cur + T::BK * (T::LDA + T::LDB);
#pragma unroll
      for (int kk = 0; kk < T::BK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        double a[T::FM], bo[FNO];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm) a[fm] = cur[kr * T::LDA + (wm * T::FM + fm) * 16 + (lane & 15)];
#pragma unroll
        for (int f = 0; f < FNO; ++f) bo[f] = so[kr * LDO + f * 16 + (lane & 15)];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
          for (int f = 0; f < FNO; ++f)
            aco[fm][f] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fm], bo[f], aco[fm][f], 0, 0, 0);
      }
      if ((s % cs) == cs - 1) {  // b complete: Ot2[p][l][a][b] += aco(a, l)
        const int b = bb0 + s / cs;
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
          for (int f = 0; f < FNO; ++f) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int a = m0 + acc_row<T>(wm, fm, lane, rr);
              const int l = f * 16 + (lane & 15);
              if (a < nv && l < no)
                unsafeAtomicAdd(&Ot2[(((int64_t)p * no + l) * nvl + a) * nvl + b], aco[fm][f][rr]);
            }
            aco[fm][f] = d4v{0.0, 0.0, 0.0, 0.0};
          }
      }
    }
    if (more) store(nxt);
    __syncthreads();
  }
  // (d, Omega1) columns
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = m0 + acc_row<T>(wm, fm, lane, rr);
        const int n = n0 + acc_col<T>(wn, fn, lane);
        if (a >= nv) continue;
        if (n < nv) unsafeAtomicAdd(&Ot2[(((int64_t)p * no + q) * nvl + a) * nvl + n], acc[fm][fn][rr]);
        else if (n == nv) unsafeAtomicAdd(&Ot1[(int64_t)p * nvl + a], acc[fm][fn][rr]);
      }
}

void launch_omega(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Ot1,
                  double* Ot2, int no, int nv, hipStream_t st) {
  typedef OCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + 1 + T::BN - 1) / T::BN;
  const int bchunk = 8;
  const int nbc = (nv + bchunk - 1) / bchunk;
  const dim3 grid(nbc * tm * tn, 6, ntri), block(T::NT);
  if (no <= 16)
    hipLaunchKernelGGL(k_omega<1>, grid, block, 0, st, cubes, b.Gv, b.Jo, b.Hs, tri, Ot1, Ot2, no, nv, bchunk, nbc, tn);
  else if (no <= 32)
    hipLaunchKernelGGL(k_omega<2>, grid, block, 0, st, cubes, b.Gv, b.Jo, b.Hs, tri, Ot1, Ot2, no, nv, bchunk, nbc, tn);
  else if (no <= 48)
    hipLaunchKernelGGL(k_omega<3>, grid, block, 0, st, cubes, b.Gv, b.Jo, b.Hs, tri, Ot1, Ot2, no, nv, bchunk, nbc, tn);
  else
    hipLaunchKernelGGL(k_omega<4>, grid, block, 0, st, cubes, b.Gv, b.Jo, b.Hs, tri, Ot1, Ot2, no, nv, bchunk, nbc, tn);
}

// FLOP of the dominant contractions and their companions, padding excluded.
double wbuild_flops(int no, int nv, const int* kinds, int n) {
  const double v = nv, o = no;
  const double term = 2.0 * v * v * v * v + 2.0 * v * v * v * o;
  double f = 0.0;
  for (int t = 0; t < n; ++t) f += (kinds[t] == TRI_DISTINCT ? 6.0 : 3.0) * term;
  return f;
}

double omega_flops(int no, int nv, const int* kinds, int n) {
  const double v = nv, o = no;
  const double perm = 2.0 * v * v * v * v + 2.0 * v * v * v + 2.0 * v * v * v * (o + 1.0);
  double f = 0.0;
  for (int t = 0; t < n; ++t) f += (kinds[t] == TRI_DISTINCT ? 6.0 : 3.0) * perm;
  return f;
}

}  // namespace cc3
