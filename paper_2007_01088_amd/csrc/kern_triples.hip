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
//            U = tau~_{pqr} read from tau~ or tau~T, one long-K GEMM over K = (b, c):
//              Ot2[p][q][a][d] += sum_bc U[a,b,c] g_{dbrc}    (columns d < nv)
//              Ot1[p][a]       += sum_bc U[a,b,c] g_{qbrc}    (column nv)
//            split over K into per-(triple, permutation, chunk) partial slabs;
//  k_reduce  adds the slabs into Ot1/Ot2 in a fixed order (deterministic, no atomics);
//  k_omega_oo (FP64 MFMA, output-stationary)  the oo and Fock terms
//              Ot2[p][l][a][b] += sum_c U[a,b,c] (delta_lq F_rc - g_{qlrc}),
//            kept transposed, OtT[p][l][b][a], so that its stores run along a.
#include <algorithm>

#include "cc3.h"
#include "cc3_device.hpp"
#include "cc3_internal.hpp"

namespace cc3 {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// cube slots of one triple's workspace
enum { SLOT_P0 = 0, SLOT_P1 = 1, SLOT_P2 = 2, SLOT_TT = 3, SLOT_TTT = 4, NSLOT = 5 };

// ---------------------------------------------------------------------------
// W build
// ---------------------------------------------------------------------------
typedef TileCfg<4, 2, 2, 4, 16> WCfg;  // 128 x 128 output plane tile, 8 wavefronts, 16 k per stage

// MODE 0: the t3 terms (t2, t2N, Gw, Go as named).  MODE 1: the L3 terms of
// Algorithm 3, C_pqr[x,y,z] = sum_d L^{xd}_{qr} g_{pydz} - sum_l L^{xy}_{lr} g_{plqz}
// (+ outer products added by the density mix), with t2 <- l2, t2N <- l2M
// (l2M[r][y][x][l] = -l2[l][r][x][y]), Gw <- Gl (Gl[p][y][z][d] = g_{pydz}) and
// Go <- Go3 (Go3[p][q][z][l] = g_{plqz}): the same segments with the roles of the
// occupied indices permuted.  Plane `plane` of triple z goes to cubes + z zs + plane ss.
template <int MODE>
__device__ __forceinline__ void wbuild_body(const double* __restrict__ t2,
                                            const double* __restrict__ t2N,
                                            const double* __restrict__ Gw,
                                            const double* __restrict__ Go,
                                            const int* __restrict__ tri,
                                            double* __restrict__ cubes, int64_t zs, int64_t ss,
                                            int pitch, int no, int nv, int tiles_m, int tiles_n,
                                            int all_terms, int bx, int by, int bz) {
  typedef WCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int tpp = tiles_m * tiles_n;
  const int y = bx / tpp;
  const int tile = bx % tpp;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const int plane = by;
  const int z = bz;
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

  // Four K segments, each a product of two row-major (row, k) operands with k contiguous:
  //   term 1: Acc[m][n] += sum_d t2[p1][q1][m][d] Gw[r1][y][n][d]       (K = nv)
  //                      + sum_l t2N[p1][y][m][l] Go[q1][r1][n][l]      (K = no)
  //   term 2: Acc[m][n] += sum_d Gw[r2][y][m][d] t2[p2][q2][n][d]       (K = nv)
  //                      + sum_l Go[q2][r2][m][l] t2N[p2][y][n][l]      (K = no)
  // with t2N[p][y][x][l] = -t2[p][l][x][y].  The row stride of a segment is its K.
  // Tile origins (row m0 / n0, k = 0) of the eight operands, as byte pointers:
  // MODE 1 takes the amplitude pair (q, r), the (v v|. .) slab of p and the (o o|o v)
  // slab of (p, q) where MODE 0 takes (p, q), r and (q, r)
  const int ax1 = MODE ? q1 : p1, bx1 = MODE ? r1 : q1, g1 = MODE ? p1 : r1;
  const int an1 = MODE ? r1 : p1, h1a = MODE ? p1 : q1, h1b = MODE ? q1 : r1;
  const int ax2 = MODE ? q2 : p2, bx2 = MODE ? r2 : q2, g2 = MODE ? p2 : r2;
  const int an2 = MODE ? r2 : p2, h2a = MODE ? p2 : q2, h2b = MODE ? q2 : r2;
  const char* A0 = (const char*)(t2 + ((int64_t)ax1 * no + bx1) * nv2 + (int64_t)m0 * nv);
  const char* B0 = (const char*)(Gw + ((int64_t)g1 * nv + y) * nv2 + (int64_t)n0 * nv);
  const char* A1 = (const char*)(t2N + ((int64_t)an1 * nv + y) * nv * no + (int64_t)m0 * no);
  const char* B1 = (const char*)(Go + ((int64_t)h1a * no + h1b) * nv * no + (int64_t)n0 * no);
  const char* A2 = (const char*)(Gw + ((int64_t)g2 * nv + y) * nv2 + (int64_t)m0 * nv);
  const char* B2 = (const char*)(t2 + ((int64_t)ax2 * no + bx2) * nv2 + (int64_t)n0 * nv);
  const char* A3 = (const char*)(Go + ((int64_t)h2a * no + h2b) * nv * no + (int64_t)m0 * no);
  const char* B3 = (const char*)(t2N + ((int64_t)an2 * nv + y) * nv * no + (int64_t)n0 * no);
  // This thread's part of every stage: k = kt and rows xt + e * RP of both tiles.  Rows
  // past nv repeat row nv - 1 (their outputs are never stored).  Loads go through buffer
  // resources built from the (uniform) stage origin with 32-bit byte offsets per lane.
  const int tid = threadIdx.x;
  constexpr int RP = T::NT / T::BK;
  const int kt = tid % T::BK, xt = tid / T::BK;
  int rowa[T::EA], rowb[T::EB];
#pragma unroll
  for (int e = 0; e < T::EA; ++e) rowa[e] = min(m0 + xt + e * RP, nv - 1) - m0;
#pragma unroll
  for (int e = 0; e < T::EB; ++e) rowb[e] = min(n0 + xt + e * RP, nv - 1) - n0;
  // swizzled LDS slots of (kt, xt + e * RP): RP is a multiple of 16, so the XOR
  // pattern of row kt only touches xt
  const int lda = kt * T::LDA + (xt ^ lds_swz<T::BK>(kt));
  const int ldb = T::BK * T::LDA + kt * T::LDB + (xt ^ lds_swz<T::BK>(kt));
  double ra[T::EA], rb[T::EB];
  int lseg = 0, lk0 = 0;  // the next stage to load
  int ks_load = 0;         // MFMA k-steps of 4 that hold data in the stage just loaded
  bool zin = true;         // this lane's k of the stage just loaded lies inside its segment
  auto fetch = [&]() {
    const char *pa, *pb;
    if (lseg == 0) { pa = A0; pb = B0; }
    else if (lseg == 1) { pa = A1; pb = B1; }
    else if (lseg == 2) { pa = A2; pb = B2; }
    else { pa = A3; pb = B3; }
    const int ld = (lseg & 1) ? no : nv;
    const BufRsrc sa = buf_rsrc(pa + lk0 * 8), sb = buf_rsrc(pb + lk0 * 8);
    const bool in = lk0 + kt < ld;                    // the segment's last stage may be partial
    const int kc = in ? kt : ld - 1 - lk0;           // k past K reads a valid element
    // The zero of k past K is applied when the stage is stored: a select here would
    // wait for the loads before the current stage's MFMAs instead of after them.
#pragma unroll
    for (int e = 0; e < T::EA; ++e) ra[e] = buf_load_f64(sa, (unsigned)(rowa[e] * ld + kc) * 8u);
#pragma unroll
    for (int e = 0; e < T::EB; ++e) rb[e] = buf_load_f64(sb, (unsigned)(rowb[e] * ld + kc) * 8u);
    zin = in;
    ks_load = min(T::BK, ld - lk0 + 3) / 4;  // a segment's last stage may be part zeros
    lk0 += T::BK;
    if (lk0 >= ld) { lk0 = 0; ++lseg; }
  };
  auto store = [&](double* st) {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) st[lda + e * RP] = zin ? ra[e] : 0.0;
#pragma unroll
    for (int e = 0; e < T::EB; ++e) st[ldb + e * RP] = zin ? rb[e] : 0.0;
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  fetch();
  store(lds);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    double* cur = lds + (s & 1) * T::STAGE;
    double* nxt = lds + ((s + 1) & 1) * T::STAGE;
    const bool more = s + 1 < nsteps;
    const int ks = ks_load;  // k-steps of the stage computed now (uniform)
    if (more) fetch();
    // as mfma_stage, skipping the k-steps of a segment's last stage that hold only zeros
#pragma unroll
    for (int kk = 0; kk < T::BK / 4; ++kk) {
      if (kk >= ks) break;
      const int kr = kk * 4 + (lane >> 4);
      const int sw = (lane & 15) ^ lds_swz<T::BK>(kr);
      double a[T::FM], b[T::FN];
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) a[fm] = cur[kr * T::LDA + (wm * T::FM + fm) * 16 + sw];
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn)
        b[fn] = cur[T::BK * T::LDA + kr * T::LDB + (wn * T::FN + fn) * 16 + sw];
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
    }
    if (more) store(nxt);
    __syncthreads();
  }

  double* out = cubes + (int64_t)z * zs + (int64_t)plane * ss + (int64_t)y * nv * pitch;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + acc_row<T>(wm, fm, lane, r);
        const int n = n0 + acc_col<T>(wn, fn, lane);
        if (m < nv && n < nv) out[(int64_t)m * pitch + n] = acc[fm][fn][r];
      }
}

template <int MODE>
__global__ __launch_bounds__(WCfg::NT) void k_wbuild(const double* __restrict__ t2,
                                                     const double* __restrict__ t2N,
                                                     const double* __restrict__ Gw,
                                                     const double* __restrict__ Go,
                                                     const int* __restrict__ tri,
                                                     double* __restrict__ cubes, int64_t zs,
                                                     int64_t ss, int pitch, int no, int nv,
                                                     int tiles_m, int tiles_n, int all_terms) {
  wbuild_body<MODE>(t2, t2N, Gw, Go, tri, cubes, zs, ss, pitch, no, nv, tiles_m, tiles_n,
                    all_terms, blockIdx.x, blockIdx.y, blockIdx.z);
}

void launch_wbuild_ex(int mode, const double* X, const double* XN, const double* G, const double* H,
                      const int* tri, int ntri, double* cubes, int64_t zs, int64_t ss, int pitch,
                      int no, int nv, bool all_terms, hipStream_t st) {
  typedef WCfg T;
  if (ntri <= 0) return;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + T::BN - 1) / T::BN;
  if (mode == 0)
    hipLaunchKernelGGL(k_wbuild<0>, dim3(nv * tm * tn, 3, ntri), dim3(T::NT), 0, st, X, XN, G, H,
                       tri, cubes, zs, ss, pitch, no, nv, tm, tn, all_terms ? 1 : 0);
  else
    hipLaunchKernelGGL(k_wbuild<1>, dim3(nv * tm * tn, 3, ntri), dim3(T::NT), 0, st, X, XN, G, H,
                       tri, cubes, zs, ss, pitch, no, nv, tm, tn, all_terms ? 1 : 0);
}

void launch_wbuild(const double* t2, const double* t2N, const Blocks& b, const int* tri, int ntri,
                   double* cubes, int no, int nv, bool all_terms, hipStream_t st) {
  const int64_t cs = cube_slot(nv);
  launch_wbuild_ex(0, t2, t2N, b.Gw, b.Go, tri, ntri, cubes, NSLOT * cs, cs, cube_pitch(nv), no,
                   nv, all_terms, st);
}

// t2N[p][y][x][l] = -t2[p][l][x][y]
__global__ void k_t2N(const double* __restrict__ t2, double* __restrict__ t2N, int no, int nv) {
  const int64_t nvl = nv, n = (int64_t)no * no * nvl * nvl;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int l = (int)(e % no), x = (int)((e / no) % nvl), y = (int)((e / (no * nvl)) % nvl);
  const int p = (int)(e / (no * nvl * nvl));
  t2N[e] = -t2[(((int64_t)p * no + l) * nvl + x) * nvl + y];
}

void launch_t2N(const double* t2, double* t2N, int no, int nv, hipStream_t st) {
  const int64_t n = (int64_t)no * no * nv * nv;
  hipLaunchKernelGGL(k_t2N, dim3(nblk(n, 256)), dim3(256), 0, st, t2, t2N, no, nv);
}

// ---------------------------------------------------------------------------
// Mix: X, tau, tau~ on the S3 orbit of an 8x8x8 block triple (A <= B <= C).
// ---------------------------------------------------------------------------
#define MT 8
#define MT3 (MT * MT * MT)
// padded LDS position of tile element (u, v, w): strides 73 and 9 keep every
// permuted access pattern of the orbit conflict-free across 8 lanes
#define TP(u, v, w) ((u) * 73 + (v) * 9 + (w))
#define TSZ 584

// the six orientations of a block triple, as positions into (A, B, C)
__host__ __device__ inline void orient(int o, int& p0, int& p1, int& p2) {
  switch (o) {
    case 0: p0 = 0; p1 = 1; p2 = 2; break;
    case 1: p0 = 0; p1 = 2; p2 = 1; break;
    case 2: p0 = 1; p1 = 0; p2 = 2; break;
    case 3: p0 = 1; p1 = 2; p2 = 0; break;
    case 4: p0 = 2; p1 = 0; p2 = 1; break;
    default: p0 = 2; p1 = 1; p2 = 0; break;
  }
}

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

// Threads per mix workgroup (MIXT, 256 or 512): each handles MIXH = 512 / MIXT of
// the 512 elements of an orientation tile.

__device__ inline double xval(const double* __restrict__ cz, int kind, int64_t nv, int a, int b,
                              int c) {
  const int64_t rp = cube_pitch((int)nv), pl = nv * rp, cs = cube_slot((int)nv);
  const double* P0 = cz + SLOT_P0 * cs;
  const double* P1 = cz + SLOT_P1 * cs;
  const double* P2 = cz + SLOT_P2 * cs;
  if (kind == TRI_DISTINCT)
    return P0[b * pl + a * rp + c] + P1[a * pl + b * rp + c] + P2[c * pl + a * rp + b];
  if (kind == TRI_IJ)  // P1 = P0, P2[c][a][b] = Q[c][a][b] + Q[c][b][a]
    return P0[b * pl + a * rp + c] + P0[a * pl + b * rp + c] + P2[c * pl + a * rp + b] +
           P2[c * pl + b * rp + a];
  // TRI_JK: P2 = P0, P1[a][b][c] = R[a][b][c] + R[a][c][b]
  return P0[b * pl + a * rp + c] + P1[a * pl + b * rp + c] + P1[a * pl + c * rp + b] +
         P0[c * pl + a * rp + b];
}

// The split-BF16 pieces of x at row `row` and K pair (kx, ky) of view v of triple z in
// YL[z][4][P][nv][Kr] (rows of pitch Kr = lp_kb_pitch(nv), the pair at lp_kb(kx, ky)).
__device__ inline void yl_put(uint16_t* YL, int P, int z, int v, int row, int kx, int ky, int nv,
                              double x) {
  const int64_t Kr = lp_kb_pitch(nv);
  uint16_t* base = YL + (((int64_t)z * 4 + v) * P * nv + row) * Kr + lp_kb(kx, ky, nv);
  const int64_t ps = (int64_t)nv * Kr;
  if (P == 2) {
    uint16_t pc[2];
    split_bf16<2>(x, pc);
    base[0] = pc[0];
    base[ps] = pc[1];
  } else {
    uint16_t pc[3];
    split_bf16<3>(x, pc);
    base[0] = pc[0];
    base[ps] = pc[1];
    base[2 * ps] = pc[2];
  }
}

// Mixed-all copies (nullable): cubesF, FP32 tau~ and tau~T, [triple][2][nv^3];
// YL, the split-BF16 k-major views of the split-BF16 Omega GEMM (k_omega_lp),
// [triple][4][piece][a][kk < Kp] with lpP pieces.
template <int MIXT>
__device__ __forceinline__ void mix_body(const double* __restrict__ eps,
                                         const int* __restrict__ tri, double* __restrict__ cubes,
                                         float* __restrict__ cubesF, uint16_t* __restrict__ YL,
                                         int lpP, int no, int nv, int bx, int by) {
  constexpr int MIXH = 512 / MIXT;
  __shared__ double Xs[6 * TSZ];
  const int z = by, ob = bx;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  const int kind = tri_kind(i, j, k);
  const int64_t nvl = nv, nv3 = nvl * nvl * nvl;
  // the padded cube rows: pitch rp, plane pl, slot cs
  const int64_t rp = cube_pitch(nv), pl = nvl * rp, cs = cube_slot(nv);
  double* cz = cubes + (int64_t)z * NSLOT * cs;
  int blk[3];
  decode_block_triple(ob, blk[0], blk[1], blk[2]);
  // With equal blocks some orientations repeat an earlier one: canon[o] is the
  // first orientation with the same block triple.  Repeats are neither loaded,
  // combined nor written; reads of a repeated tile go to its first copy.
  int canon[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    canon[o] = o;
#pragma unroll
    for (int o2 = 4; o2 >= 0; --o2) {
      if (o2 >= o) continue;
      int r0, r1, r2;
      orient(o2, r0, r1, r2);
      if (blk[r0] == blk[q0] && blk[r1] == blk[q1] && blk[r2] == blk[q2]) canon[o] = o2;
    }
  }
  const double eijk = eps[i] + eps[j] + eps[k];
  const double* P0 = cz + SLOT_P0 * cs;
  const double* P1 = cz + SLOT_P1 * cs;
  const double* P2 = cz + SLOT_P2 * cs;
  const int t = threadIdx.x;
  // 1. X on the orbit.  Each orientation tile is summed in up to three passes
  //    whose thread mapping makes the contiguous index of the cubes read in
  //    that pass the fastest one (c, b, then a).
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int A0 = blk[q0] * MT, B0 = blk[q1] * MT, C0 = blk[q2] * MT;
#pragma unroll
    for (int h = 0; h < MIXH; ++h) {
      const int e = t + MIXT * h;
      const int u = e >> 6, v = (e >> 3) & 7, w = e & 7;  // pass 0: c fastest
      const int a = A0 + u, b = B0 + v, c = C0 + w;
      double x = 0.0;
      if (a < nv && b < nv && c < nv)
        x = P0[b * pl + a * rp + c] + (kind == TRI_IJ ? P0 : P1)[a * pl + b * rp + c];
      Xs[o * TSZ + TP(u, v, w)] = x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int A0 = blk[q0] * MT, B0 = blk[q1] * MT, C0 = blk[q2] * MT;
#pragma unroll
    for (int h = 0; h < MIXH; ++h) {
      const int e = t + MIXT * h;
      const int u = e >> 6, w = (e >> 3) & 7, v = e & 7;  // pass 1: b fastest
      const int a = A0 + u, b = B0 + v, c = C0 + w;
      if (a < nv && b < nv && c < nv) {
        double x;
        if (kind == TRI_JK) x = P1[a * pl + c * rp + b] + P0[c * pl + a * rp + b];
        else x = P2[c * pl + a * rp + b];
        Xs[o * TSZ + TP(u, v, w)] += x;
      }
    }
  }
  if (kind == TRI_IJ) {
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      if (canon[o] != o) continue;
      int q0, q1, q2;
      orient(o, q0, q1, q2);
      const int A0 = blk[q0] * MT, B0 = blk[q1] * MT, C0 = blk[q2] * MT;
#pragma unroll
      for (int h = 0; h < MIXH; ++h) {
        const int e = t + MIXT * h;
        const int v = e >> 6, w = (e >> 3) & 7, u = e & 7;  // pass 2: a fastest
        const int a = A0 + u, b = B0 + v, c = C0 + w;
        if (a < nv && b < nv && c < nv) Xs[o * TSZ + TP(u, v, w)] += P2[c * pl + b * rp + a];
      }
    }
  }
  __syncthreads();
  // 2. tau~ on the orbit, held in registers until every thread has read X
  double tt[6][MIXH];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int A0 = blk[q0] * MT, B0 = blk[q1] * MT, C0 = blk[q2] * MT;
    const int o_acb = canon[orient_of(q0, q2)], o_cba = canon[orient_of(q2, q1)];
    const int o_bac = canon[orient_of(q1, q0)], o_bca = canon[orient_of(q1, q2)];
    const int o_cab = canon[orient_of(q2, q0)];
#pragma unroll
    for (int h = 0; h < MIXH; ++h) {
      const int e = t + MIXT * h;
      const int u = e >> 6, v = (e >> 3) & 7, w = e & 7;
      const int a = A0 + u, b = B0 + v, c = C0 + w;
      double val = 0.0;
      if (a < nv && b < nv && c < nv) {
        // X at permuted virtual labels: (a,c,b), (c,b,a), (b,a,c), (b,c,a), (c,a,b)
        const double x_abc = Xs[o * TSZ + TP(u, v, w)];
        const double x_acb = Xs[o_acb * TSZ + TP(u, w, v)];
        const double x_cba = Xs[o_cba * TSZ + TP(w, v, u)];
        const double x_bac = Xs[o_bac * TSZ + TP(v, u, w)];
        const double x_bca = Xs[o_bca * TSZ + TP(v, w, u)];
        const double x_cab = Xs[o_cab * TSZ + TP(w, u, v)];
        const double D = eps[no + a] + eps[no + b] + eps[no + c] - eijk;
        val = -(4.0 * x_abc - 2.0 * x_acb - 2.0 * x_cba - 2.0 * x_bac + x_bca + x_cab) / D;
      }
      tt[o][h] = val;
    }
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
#pragma unroll
    for (int h = 0; h < MIXH; ++h) {
      const int e = t + MIXT * h;
      Xs[o * TSZ + TP(e >> 6, (e >> 3) & 7, e & 7)] = tt[o][h];
    }
  }
  __syncthreads();
  // 3. write tau~[a][b][c] (w fastest) and tau~T[a][c][b] (v fastest)
  double* TT = cz + SLOT_TT * cs;
  double* TTT = cz + SLOT_TTT * cs;
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int A0 = blk[q0] * MT, B0 = blk[q1] * MT, C0 = blk[q2] * MT;
#pragma unroll
    for (int h = 0; h < MIXH; ++h) {
      const int e = t + MIXT * h;
      {
        const int u = e >> 6, v = (e >> 3) & 7, w = e & 7;
        const int a = A0 + u, b = B0 + v, c = C0 + w;
        if (a < nv && b < nv && c < nv) {
          const double x = Xs[o * TSZ + TP(u, v, w)];
          TT[(a * nvl + b) * rp + c] = x;
          if (cubesF) cubesF[(int64_t)z * 2 * nv3 + (a * nvl + b) * nvl + c] = (float)x;
          if (YL) {  // view 0 at [a][(b, c)], view 1 at [b][(a, c)]
            yl_put(YL, lpP, z, 0, a, b, c, nv, x);
            yl_put(YL, lpP, z, 1, b, a, c, nv, x);
          }
        }
      }
      {
        const int u = e >> 6, w = (e >> 3) & 7, v = e & 7;
        const int a = A0 + u, b = B0 + v, c = C0 + w;
        if (a < nv && b < nv && c < nv) {
          const double x = Xs[o * TSZ + TP(u, v, w)];
          TTT[(a * nvl + c) * rp + b] = x;
          if (cubesF) cubesF[((int64_t)z * 2 + 1) * nv3 + (a * nvl + c) * nvl + b] = (float)x;
          if (YL) {  // view 2 at [c][(a, b)], view 3 at [a][(c, b)]
            yl_put(YL, lpP, z, 2, c, a, b, nv, x);
            yl_put(YL, lpP, z, 3, a, c, b, nv, x);
          }
        }
      }
    }
  }
}

template <int MIXT>
__global__ __launch_bounds__(MIXT) void k_mix(const double* __restrict__ eps,
                                             const int* __restrict__ tri,
                                             double* __restrict__ cubes, float* __restrict__ cubesF,
                                             uint16_t* __restrict__ YL, int lpP, int no, int nv) {
  mix_body<MIXT>(eps, tri, cubes, cubesF, YL, lpP, no, nv, blockIdx.x, blockIdx.y);
}

void launch_mix(const double* eps, const int* tri, int ntri, double* cubes, float* cubesF,
                void* YL, int lpP, int no, int nv, hipStream_t st) {
  const int nb = (nv + MT - 1) / MT;
  const int nbt = nb * (nb + 1) * (nb + 2) / 6;
  // 512 threads, one element per thread and orientation; the form that also writes
  // the split-BF16 views of tau~ runs with 256 (two elements each), which measured
  // faster for it at nv = 250
  if (YL)
    hipLaunchKernelGGL(k_mix<256>, dim3(nbt, ntri), dim3(256), 0, st, eps, tri, cubes, cubesF,
                       (uint16_t*)YL, lpP, no, nv);
  else
    hipLaunchKernelGGL(k_mix<512>, dim3(nbt, ntri), dim3(512), 0, st, eps, tri, cubes, cubesF,
                       (uint16_t*)YL, lpP, no, nv);
}

// ---------------------------------------------------------------------------
// Mix of the transition-density loop (Algorithm 3).  Cubes are slot-major,
// cubes[slot][z][cube] (slot stride ss; each cube nv x nv rows at the padded pitch
// cube_pitch), so that each slot of a batch is one contiguous run of cubes.  LMODE false: from the t3 planes, tau = -X/eps and
// tau~ (the contravariant combination) into slots D3_TAU, D3_TAUC.  LMODE true:
// from the L3 planes plus the outer-product terms of the L3 statement,
//   sum over the six simultaneous permutations (p,q,r; x,y,z) of (i,j,k; a,b,c) of
//   L^x_p g_{qyrz} + L^{xy}_{pq} F_{rz},
// L = X / (omega - eps) and its contravariant L~ into slot D3_LC.
// Same S3-orbit tiling of 8^3 virtual blocks as k_mix; outputs are written in
// [a][b][c] order straight from the orientation tiles.
// ---------------------------------------------------------------------------
__device__ inline double l3_outer(const double* __restrict__ l1, const double* __restrict__ l2,
                                  const double* __restrict__ Jo, const double* __restrict__ F,
                                  int no, int64_t nv, int i, int j, int k, int a, int b, int c) {
  auto term = [&](int p, int q, int r, int x, int y, int z) {
    return l1[(int64_t)p * nv + x] * Jo[(((int64_t)q * no + r) * nv + y) * nv + z] +
           l2[(((int64_t)p * no + q) * nv + x) * nv + y] * F[(int64_t)r * nv + z];
  };
  return term(i, j, k, a, b, c) + term(j, i, k, b, a, c) + term(k, j, i, c, b, a) +
         term(i, k, j, a, c, b) + term(j, k, i, b, c, a) + term(k, i, j, c, a, b);
}

template <bool LMODE>
__global__ __launch_bounds__(512) void k_mix3(const double* __restrict__ eps,
                                             const int* __restrict__ tri,
                                             double* __restrict__ cubes, int64_t ss, double omega,
                                             const double* __restrict__ l1,
                                             const double* __restrict__ l2,
                                             const double* __restrict__ Jo,
                                             const double* __restrict__ F, int no, int nv) {
  __shared__ double Xs[6 * TSZ];
  const int z = blockIdx.y, ob = blockIdx.x;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  const int kind = tri_kind(i, j, k);
  const int64_t nvl = nv;
  // the padded cube rows: pitch rp, plane pl, cube cs
  const int64_t rp = cube_pitch(nv), pl = nvl * rp, cs = cube_slot(nv);
  const double* P0 = cubes + D3_P0 * ss + (int64_t)z * cs;
  const double* P1 = cubes + D3_P1 * ss + (int64_t)z * cs;
  const double* P2 = cubes + D3_P2 * ss + (int64_t)z * cs;
  int blk[3];
  decode_block_triple(ob, blk[0], blk[1], blk[2]);
  int canon[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    canon[o] = o;
#pragma unroll
    for (int o2 = 4; o2 >= 0; --o2) {
      if (o2 >= o) continue;
      int r0, r1, r2;
      orient(o2, r0, r1, r2);
      if (blk[r0] == blk[q0] && blk[r1] == blk[q1] && blk[r2] == blk[q2]) canon[o] = o2;
    }
  }
  const int t = threadIdx.x;
  const int u = t >> 6, v = (t >> 3) & 7, w = t & 7;
  // X on the orbit: the plane sums of k_mix (c, b, then a fastest), plus the outer
  // products in the L3 form
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int a = blk[q0] * MT + u, b = blk[q1] * MT + v, c = blk[q2] * MT + w;
    double x = 0.0;
    if (a < nv && b < nv && c < nv) {
      x = P0[b * pl + a * rp + c] + (kind == TRI_IJ ? P0 : P1)[a * pl + b * rp + c];
      if (LMODE) x += l3_outer(l1, l2, Jo, F, no, nvl, i, j, k, a, b, c);
    }
    Xs[o * TSZ + TP(u, v, w)] = x;
  }
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int uu = t >> 6, ww = (t >> 3) & 7, vv = t & 7;  // b fastest
    const int a = blk[q0] * MT + uu, b = blk[q1] * MT + vv, c = blk[q2] * MT + ww;
    if (a < nv && b < nv && c < nv) {
      double x;
      if (kind == TRI_JK) x = P1[a * pl + c * rp + b] + P0[c * pl + a * rp + b];
      else x = P2[c * pl + a * rp + b];
      Xs[o * TSZ + TP(uu, vv, ww)] += x;
    }
  }
  if (kind == TRI_IJ) {
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      if (canon[o] != o) continue;
      int q0, q1, q2;
      orient(o, q0, q1, q2);
      const int vv = t >> 6, ww = (t >> 3) & 7, uu = t & 7;  // a fastest
      const int a = blk[q0] * MT + uu, b = blk[q1] * MT + vv, c = blk[q2] * MT + ww;
      if (a < nv && b < nv && c < nv) Xs[o * TSZ + TP(uu, vv, ww)] += P2[c * pl + b * rp + a];
    }
  }
  __syncthreads();
  // the denominators and the contravariant combination; outputs in [a][b][c] order,
  // with zeros in the padding columns c >= nv of each row (the Gram contraction runs
  // over whole padded cubes)
  const double eijk = eps[i] + eps[j] + eps[k];
  double* outC = cubes + (LMODE ? D3_LC : D3_TAUC) * ss + (int64_t)z * cs;
  double* outT = cubes + D3_TAU * ss + (int64_t)z * cs;
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    if (canon[o] != o) continue;
    int q0, q1, q2;
    orient(o, q0, q1, q2);
    const int a = blk[q0] * MT + u, b = blk[q1] * MT + v, c = blk[q2] * MT + w;
    if (!(a < nv && b < nv)) continue;
    if (c >= nv) {  // a padding column (c < rp: the blocks cover exactly rp values)
      const int64_t e = (a * nvl + b) * rp + c;
      outC[e] = 0.0;
      if (!LMODE) outT[e] = 0.0;
      continue;
    }
    const int o_acb = canon[orient_of(q0, q2)], o_cba = canon[orient_of(q2, q1)];
    const int o_bac = canon[orient_of(q1, q0)], o_bca = canon[orient_of(q1, q2)];
    const int o_cab = canon[orient_of(q2, q0)];
    const double x_abc = Xs[o * TSZ + TP(u, v, w)];
    const double x_acb = Xs[o_acb * TSZ + TP(u, w, v)];
    const double x_cba = Xs[o_cba * TSZ + TP(w, v, u)];
    const double x_bac = Xs[o_bac * TSZ + TP(v, u, w)];
    const double x_bca = Xs[o_bca * TSZ + TP(v, w, u)];
    const double x_cab = Xs[o_cab * TSZ + TP(w, u, v)];
    const double D = eps[no + a] + eps[no + b] + eps[no + c] - eijk - (LMODE ? omega : 0.0);
    const int64_t e = (a * nvl + b) * rp + c;
    outC[e] = -(4.0 * x_abc - 2.0 * x_acb - 2.0 * x_cba - 2.0 * x_bac + x_bca + x_cab) / D;
    if (!LMODE) outT[e] = -x_abc / D;
  }
}

void launch_mix3(bool lmode, const double* eps, const int* tri, int ntri, double* cubes, int64_t ss,
                 double omega, const double* l1, const double* l2, const double* Jo,
                 const double* F, int no, int nv, hipStream_t st) {
  if (ntri <= 0) return;
  const int nb = (nv + MT - 1) / MT;
  const int nbt = nb * (nb + 1) * (nb + 2) / 6;
  if (lmode)
    hipLaunchKernelGGL(k_mix3<true>, dim3(nbt, ntri), dim3(512), 0, st, eps, tri, cubes, ss,
                       omega, l1, l2, Jo, F, no, nv);
  else
    hipLaunchKernelGGL(k_mix3<false>, dim3(nbt, ntri), dim3(512), 0, st, eps, tri, cubes, ss,
                       0.0, l1, l2, Jo, F, no, nv);
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
// Omega contraction: the vv term and Omega1
// ---------------------------------------------------------------------------
// One (triple, permutation) GEMM over the flattened K = (b, c), K = nv^2:
//   columns n < nv : Ot2[p][q][a][n] += sum_bc U[a,b,c] g_{nbrc}
//   column  n = nv : Ot1[p][a]       += sum_bc U[a,b,c] g_{qbrc}
// Both column kinds are rows of one block G[r][n'][.][.] (n' < nv: g_{n'brc};
// n' = nv + l: g_{lbrc}), stored once with K in (b, c) order (Gbc) and once in
// (c, b) order (Gcb).  Each of the six views U_pi of the contravariant cubes
// (TT[x][y][z] = tau~[x][y][z], TTT[x][y][z] = tau~[x][z][y]) is affine in K in
// one of the two orders:
//   pi 0: tau~[a][b][c] = TT[a][(b,c)]      k contiguous (within the padded rows)
//   pi 3: tau~[a][c][b] = TTT[a][(b,c)]
//   pi 1: tau~[b][a][c] = TTT[(b,c)][a]     a contiguous, k stride: the row pitch
//   pi 5: tau~[b][c][a] = TT[(b,c)][a]
//   pi 2: tau~[c][b][a] = TT[(c,b)][a]      the same, K in (c, b) order
//   pi 4: tau~[c][a][b] = TTT[(c,b)][a]
// so every permutation is a plain long-K GEMM.  K is split into chunks of whole
// LDS stages; each chunk writes a partial slab Pvv[z][pi][chunk][a][n] (n <= nv)
// that k_reduce sums in a fixed order.  128 x 128 tiles on 8 wavefronts of
// 32 x 64, 16 k per LDS stage, two workgroups per CU.
// The same GEMM runs on FP64 MFMA (E = double) or, for the "mixed-all" form, on
// FP32 MFMA over FP32 copies of the cubes and of Gbc / Gcb (E = float), with the
// products of each K chunk summed in FP32 and the chunks summed in FP64 by k_reduce.
typedef TileCfg<4, 2, 2, 4, 16> OCfg;
typedef float f4v_ __attribute__((ext_vector_type(4)));

template <class E>
struct OmegaAcc;
template <>
struct OmegaAcc<double> {
  typedef d4v V;
  static __device__ V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ double load(BufRsrc r, unsigned off) { return buf_load_f64(r, off); }
  // D[row][col] of the 16x16x4 FP64 MFMA: row = lane/16 + 4 r
  static __device__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct OmegaAcc<float> {
  typedef f4v_ V;
  static __device__ V mfma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ float load(BufRsrc r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  }
  // D[row][col] of the 16x16x4 FP32 MFMA: row = 4 (lane/16) + r
  static __device__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// cubes: the batch's cube slots, nslot per triple, the first of them slot0 (the
// FP64 cubes hold all five slots; the FP32 copies only TT and TTT)
template <class E>
__device__ __forceinline__ void omega_body(const E* __restrict__ cubes, int nslot, int slot0,
                                           const E* __restrict__ Gbc, const E* __restrict__ Gcb,
                                           const int* __restrict__ tri, double* __restrict__ Pvv,
                                           int no, int nv, int nchunks, int tiles_n, int bx,
                                           int by, int bz) {
  typedef OCfg T;
  typedef OmegaAcc<E> M;
  constexpr unsigned ES = sizeof(E);
  __shared__ E lds[T::LDS_DOUBLES];
  const int pi = by, z = bz;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  if (!perm_active(tri_kind(i, j, k), pi)) return;
  int p, q, r;
  perm_pqr(pi, i, j, k, p, q, r);
  const int ch = bx % nchunks, tile = bx / nchunks;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  const int64_t nvl = nv, nv2 = nvl * nvl, nv3 = nv2 * nvl;
  const int K = nv * nv;
  const int S = (K + T::BK - 1) / T::BK;
  const int s0 = (int)((int64_t)ch * S / nchunks), s1 = (int)((int64_t)(ch + 1) * S / nchunks);
  if (s0 >= s1) return;  // nchunks <= S, so never taken
  const bool cb = (pi == 2 || pi == 4);
  const bool amaj = !(pi == 0 || pi == 3);  // a contiguous, k stride pp
  const int slot = (pi == 1 || pi == 3 || pi == 4) ? SLOT_TTT : SLOT_TT;
  // the FP64 cubes keep padded rows (pitch pp, slot css); the FP32 copies do not
  const int pp = (ES == 8) ? cube_pitch(nv) : nv;
  const int64_t css = (ES == 8) ? cube_slot(nv) : nv3;
  const E* U = cubes + ((int64_t)z * nslot + slot - slot0) * css;
  const E* G = (cb ? Gcb : Gbc) + (int64_t)r * (nv + no) * nv2;
  const int ask = amaj ? pp : 1;  // k stride of A in elements (within a padded row for !amaj)
  // tile origins (k = 0) of the two operands; the A rows of the views with k
  // contiguous are nv padded rows (b, .) apart: nv * pp elements
  const E* A0 = amaj ? U + m0 : U + (int64_t)m0 * nv * pp;
  const E* B0 = G + (int64_t)n0 * K;

  // Per-thread part of every stage.  A: element e at (row/column x_e, k_e) of the
  // stage, global byte offset aoff[e] plus that of k_e from the stage origin (k_e ask
  // elements, or for k = (b, c) in padded rows the columns c past nv skipped), LDS
  // slot alds[e].  Rows past nv repeat row nv - 1 (their outputs are never stored).
  // B rows n < nv are G rows n; rows n >= nv (only in the last column tile) read the
  // Omega1 row nv + q.  Offsets are relative to the tile origin: below 191 rows of
  // stride nv * pp <= 2^20, so below 2^31 bytes.
  const int tid = threadIdx.x;
  constexpr int RP = T::NT / T::BK;  // k-fast mapping: 32 rows per element step
  constexpr int KP = T::NT / T::BM;  // a-fast mapping: 4 k per element step
  unsigned aoff[T::EA], boff[T::EB];
  int ak[T::EA], alds[T::EA], blds[T::EB];
  const int kt = tid % T::BK, xt = tid / T::BK;
  if (amaj) {
    const int x = tid % T::BM, k0t = tid / T::BM;
    const unsigned xc = (unsigned)(min(m0 + x, nv - 1) - m0);
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      ak[e] = k0t + e * KP;
      aoff[e] = xc * ES;
      alds[e] = lds_idx<T::BK>(ak[e], x, T::LDA);
    }
  } else {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      ak[e] = kt;
      aoff[e] = (unsigned)(min(m0 + xt + e * RP, nv - 1) - m0) * (unsigned)(nv * pp) * ES;
      alds[e] = lds_idx<T::BK>(kt, xt + e * RP, T::LDA);
    }
  }
#pragma unroll
  for (int e = 0; e < T::EB; ++e) {
    const int n = n0 + xt + e * RP;
    boff[e] = (unsigned)((n < nv ? n : nv + q) - n0) * (unsigned)K * ES;
    blds[e] = T::BK * T::LDA + lds_idx<T::BK>(kt, xt + e * RP, T::LDB);
  }
  const unsigned ask8 = (unsigned)ask * ES;
  E ra[T::EA], rb[T::EB];
  // which loaded elements lie inside K (bit e for A, one flag for B); the zero of the
  // others is applied at the LDS store, after the current stage's MFMAs, so that the
  // loads stay in flight during them
  unsigned amask = ~0u;
  bool inb = true;
  auto fetch = [&](int s) {
    const int k0 = s * T::BK;
    const BufRsrc sb = buf_rsrc(B0 + k0);
    const int kl = K - 1 - k0;  // last valid k of this stage (only the last stage is partial)
    amask = 0u;
    if (amaj) {
      const BufRsrc sa = buf_rsrc(A0 + (int64_t)k0 * ask);
#pragma unroll
      for (int e = 0; e < T::EA; ++e) {
        const bool in = ak[e] <= kl;
        const int kc = in ? ak[e] : kl;  // k past K reads a valid element
        ra[e] = M::load(sa, aoff[e] + (unsigned)kc * ask8);
        amask |= in ? (1u << e) : 0u;
      }
    } else {
      // k = b nv + c lies at b pp + c: the stage starts at (b0, c0), and the lane's k
      // (the same for all its elements) skips pp - nv columns per row end it passes
      const int b0 = k0 / nv, c0 = k0 - b0 * nv;
      const BufRsrc sa = buf_rsrc(A0 + (int64_t)b0 * pp + c0);
      const bool in = kt <= kl;
      const int kc = in ? kt : kl;  // k past K reads a valid element
      const unsigned ko =
          (unsigned)(kc + (ES == 8 && pp != nv ? (c0 + kc) / nv * (pp - nv) : 0)) * ES;
#pragma unroll
      for (int e = 0; e < T::EA; ++e) {
        ra[e] = M::load(sa, aoff[e] + ko);
        amask |= in ? (1u << e) : 0u;
      }
    }
    inb = kt <= kl;
    const unsigned kb = (unsigned)(inb ? kt : kl) * ES;
#pragma unroll
    for (int e = 0; e < T::EB; ++e) rb[e] = M::load(sb, boff[e] + kb);
  };
  auto store = [&](E* st) {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) st[alds[e]] = ((amask >> e) & 1u) ? ra[e] : E(0);
#pragma unroll
    for (int e = 0; e < T::EB; ++e) st[blds[e]] = inb ? rb[e] : E(0);
  };
  typename M::V acc[T::FM][T::FN];
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn) acc[fm][fn] = typename M::V{0, 0, 0, 0};
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  fetch(s0);
  store(lds);
  __syncthreads();
  for (int s = s0; s < s1; ++s) {
    E* cur = lds + ((s - s0) & 1) * T::STAGE;
    E* nxt = lds + ((s - s0 + 1) & 1) * T::STAGE;
    const bool more = s + 1 < s1;
    if (more) fetch(s + 1);
    // lane supplies A[m = l%16][k = l/16] and B[k = l/16][n = l%16] to each MFMA
#pragma unroll
    for (int kk = 0; kk < T::BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      const int sw = (lane & 15) ^ lds_swz<T::BK>(kr);
      E a[T::FM], b[T::FN];
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) a[fm] = cur[kr * T::LDA + (wm * T::FM + fm) * 16 + sw];
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn)
        b[fn] = cur[T::BK * T::LDA + kr * T::LDB + (wn * T::FN + fn) * 16 + sw];
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < T::FN; ++fn) acc[fm][fn] = M::mfma(a[fm], b[fn], acc[fm][fn]);
    }
    if (more) store(nxt);
    __syncthreads();
  }
  const int NV1 = nv + 1;
  double* pvv = Pvv + (((int64_t)z * 6 + pi) * nchunks + ch) * nvl * NV1;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = m0 + (wm * T::FM + fm) * 16 + M::row(lane, rr);
        const int n = n0 + acc_col<T>(wn, fn, lane);
        if (a < nv && n <= nv) pvv[(int64_t)a * NV1 + n] = (double)acc[fm][fn][rr];
      }
}

template <class E>
__global__ __launch_bounds__(OCfg::NT) void k_omega(const E* __restrict__ cubes, int nslot,
                                                    int slot0, const E* __restrict__ Gbc,
                                                    const E* __restrict__ Gcb,
                                                    const int* __restrict__ tri,
                                                    double* __restrict__ Pvv, int no, int nv,
                                                    int nchunks, int tiles_n) {
  omega_body<E>(cubes, nslot, slot0, Gbc, Gcb, tri, Pvv, no, nv, nchunks, tiles_n, blockIdx.x,
                blockIdx.y, blockIdx.z);
}

// The (triple, permutation) pairs of a batch whose first occupied index is p, in
// batch order (triple, then permutation): lz = 6 z + pi, lqr = q no + r; at most two
// per triple, so at most 2 * MAX_BATCH.  Every thread of the workgroup calls it (it
// holds barriers); cz is LDS scratch of MAX_BATCH + 1 ints.  Returns the count.
#define PLIST_MAX (2 * MAX_BATCH)
__device__ inline int pairs_with_p(const int* __restrict__ tri, int ntri, int p, int no, int* lz,
                                   int* lqr, int* cz) {
  if (ntri <= 8) {  // a short batch: one thread, one barrier
    if (threadIdx.x == 0) {
      int n = 0;
      for (int z = 0; z < ntri; ++z) {
        const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
        const int kind = tri_kind(i, j, k);
        for (int pi = 0; pi < 6; ++pi) {
          if (!perm_active(kind, pi)) continue;
          int pp, q, r;
          perm_pqr(pi, i, j, k, pp, q, r);
          if (pp != p) continue;
          lz[n] = z * 6 + pi;
          lqr[n] = q * no + r;
          ++n;
        }
      }
      cz[MAX_BATCH] = n;
    }
    __syncthreads();
    return cz[MAX_BATCH];
  }
  // the number of permutations with first index p of each triple (at most two)
  for (int z = threadIdx.x; z < ntri; z += blockDim.x) {
    const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
    const int kind = tri_kind(i, j, k);
    int c = 0;
    for (int pi = 0; pi < 6; ++pi) {
      if (!perm_active(kind, pi)) continue;
      int pp, q, r;
      perm_pqr(pi, i, j, k, pp, q, r);
      c += pp == p;
    }
    cz[z] = c;
  }
  __syncthreads();
  // exclusive prefix sums of the counts (wavefront 0, 64 triples at a time)
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < ntri; base += 64) {
      const int z = base + lane;
      const int v = z < ntri ? cz[z] : 0;
      int incl = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
      }
      if (z < ntri) cz[z] = carry + incl - v;
      carry += __shfl(incl, 63);
    }
    if (lane == 0) cz[MAX_BATCH] = carry;
  }
  __syncthreads();
  for (int z = threadIdx.x; z < ntri; z += blockDim.x) {
    const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
    const int kind = tri_kind(i, j, k);
    int at = cz[z];
    for (int pi = 0; pi < 6; ++pi) {
      if (!perm_active(kind, pi)) continue;
      int pp, q, r;
      perm_pqr(pi, i, j, k, pp, q, r);
      if (pp != p) continue;
      if (at < PLIST_MAX) {
        lz[at] = z * 6 + pi;
        lqr[at] = q * no + r;
      }
      ++at;
    }
  }
  const int n = min(cz[MAX_BATCH], PLIST_MAX);
  __syncthreads();
  return n;
}

// The view of U_pi[a, b, c] at fixed b as a strided (a, c) matrix: base + b * sbb, (sm, sk),
// in the cubes [x][y][z] with the row pitch rp (x stride nv rp, y stride rp).
__device__ inline void u_view(int pi, int nv, int rp, int& slot, int& sbb, int& sm, int& sk) {
  const int pl = nv * rp;
  switch (pi) {
    case 0: slot = SLOT_TT; sbb = rp; sm = pl; sk = 1; break;    // tau~[a][b][c]
    case 1: slot = SLOT_TT; sbb = pl; sm = rp; sk = 1; break;    // tau~[b][a][c]
    case 2: slot = SLOT_TT; sbb = rp; sm = 1; sk = pl; break;    // tau~[c][b][a]
    case 3: slot = SLOT_TTT; sbb = rp; sm = pl; sk = 1; break;   // tau~T[a][b][c]
    case 4: slot = SLOT_TTT; sbb = rp; sm = 1; sk = pl; break;   // tau~T[c][b][a]
    default: slot = SLOT_TT; sbb = pl; sm = 1; sk = rp; break;   // tau~[b][c][a]
  }
}

// ---------------------------------------------------------------------------
// Omega contraction: the oo and Fock terms, output-stationary
// ---------------------------------------------------------------------------
// One workgroup of 4 wavefronts per (p, pair of b, 64-wide tile of a) sums, over
// the batch's pairs with that p in batch order,
//   OtT[p][l][b][a] += sum_c Hs[q][r][c][l] U[a,b,c]      (l < no)
// (Hs[q][r][c][l] = delta_lq F_rc - g_{qlrc}) and adds the sum into OtT
// (read-modify-write; successive batches are ordered by the caller).  Wavefront w
// owns the 16 columns a0 = tile + 16 w of both b and every row l (FNO blocks of
// 16), as D[l][a] of the FP64 MFMA with A = Hs, B = U.  The kernel streams U once
// per pair and is bound by the memory pipeline, so there are no workgroup
// barriers in the loop: the next step's loads are in flight during the current
// step's MFMAs, and the Hs fragments serve both b.  Within a 16-c step, lane
// group kq = lane / 16 feeds c = c0 + 4 kq + t to MFMA t (the same order on both
// operands, which leaves the sum unchanged).  Views with a contiguous are loaded
// in the MFMA layout directly (16 consecutive a per row of c); views with c
// contiguous are loaded along c (4 rows of 16 consecutive c per instruction) and
// transposed through a wavefront-private LDS tile.
template <int FNO>
__device__ __forceinline__ void omega_oo_body(const double* __restrict__ cubes,
                                              const double* __restrict__ Hs,
                                              const int* __restrict__ tri, int ntri,
                                              double* __restrict__ OtT, int no, int nv,
                                              int tiles_a, int bx, int by) {
  constexpr int NB = 2;
  __shared__ int lz[PLIST_MAX], lqr[PLIST_MAX], cz[MAX_BATCH + 1];
  int cnt;
  __shared__ double lt[4][NB][16][17];  // per wavefront: 16 rows a x 16 c (+1 pad)
  const int p = by;
  const int bp = bx / tiles_a;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a0 = (bx % tiles_a) * 64 + 16 * wave;
  cnt = pairs_with_p(tri, ntri, p, no, lz, lqr, cz);
  const int n = cnt;
  if (n == 0 || a0 >= nv) return;  // no workgroup barrier follows
  const int m = lane & 15, kq = lane >> 4;
  int bb[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) bb[j] = min(NB * bp + j, nv - 1);
  const int64_t nvl = nv, nv2 = nvl * nvl;
  d4v acc[NB][FNO];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int f = 0; f < FNO; ++f) acc[j][f] = d4v{0.0, 0.0, 0.0, 0.0};
  // flattened (pair, 16-c step) loop with the next step's loads issued before
  // the current step's MFMAs
  const int cs = (nv + 15) / 16;
  const int nit = n * cs;
  // Elements with c past nv load a valid element (c clamped) and are zeroed when they
  // are used (cm: bit i or tt set for c < nv), so that the next step's loads stay in
  // flight over the current step's MFMAs.
  double u[2][NB][4], h[2][FNO][4];
  bool cc1[2];
  unsigned cm1[2];
  auto load = [&](int it, double (&uu)[NB][4], double (&hh)[FNO][4], bool& ccont,
                  unsigned& cm) {
    const int t = it / cs, c0 = (it - t * cs) * 16;
    const int zp = lz[t], zz = zp / 6, pi = zp % 6;
    int slot, sbb, sm, sk;
    u_view(pi, nv, cube_pitch(nv), slot, sbb, sm, sk);
    const double* ub = cubes + ((int64_t)zz * NSLOT + slot) * cube_slot(nv);
    ccont = (sk == 1);
    if (ccont) {  // element i: row a0 + 4 i + kq, c = c0 + m
      const int c = c0 + m;
      const int cc = min(c, nv - 1);
      cm = c < nv ? 15u : 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = min(a0 + 4 * i + kq, nv - 1);
#pragma unroll
        for (int j = 0; j < NB; ++j) uu[j][i] = ub[(int64_t)row * sm + (int64_t)bb[j] * sbb + cc];
      }
    } else {  // element tt: row a0 + m, c = c0 + 4 kq + tt
      const int64_t ra = (int64_t)min(a0 + m, nv - 1);
      cm = 0u;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int c = c0 + 4 * kq + tt;
        const int cc = min(c, nv - 1);
        cm |= c < nv ? 1u << tt : 0u;
#pragma unroll
        for (int j = 0; j < NB; ++j) uu[j][tt] = ub[ra + (int64_t)bb[j] * sbb + (int64_t)cc * sk];
      }
    }
    const double* hb = Hs + (int64_t)lqr[t] * no * nvl;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const int cc = min(c0 + 4 * kq + tt, nv - 1);
#pragma unroll
      for (int f = 0; f < FNO; ++f) hh[f][tt] = hb[(int64_t)cc * no + min(16 * f + m, no - 1)];
    }
  };
  auto mma = [&](const double (&uu)[NB][4], const double (&hh)[FNO][4], bool ccont, unsigned cm) {
    double x[NB][4];
    if (ccont) {  // transpose through this wavefront's LDS tile
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) lt[wave][j][4 * i + kq][m] = cm ? uu[j][i] : 0.0;
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) x[j][tt] = lt[wave][j][m][4 * kq + tt];
      __builtin_amdgcn_wave_barrier();
    } else {
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) x[j][tt] = ((cm >> tt) & 1u) ? uu[j][tt] : 0.0;
    }
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int f = 0; f < FNO; ++f)
          acc[j][f] = __builtin_amdgcn_mfma_f64_16x16x4f64(hh[f][tt], x[j][tt], acc[j][f], 0, 0, 0);
  };
  load(0, u[0], h[0], cc1[0], cm1[0]);
  for (int it = 0; it < nit; it += 2) {
    if (it + 1 < nit) load(it + 1, u[1], h[1], cc1[1], cm1[1]);
    mma(u[0], h[0], cc1[0], cm1[0]);
    if (it + 1 < nit) {
      if (it + 2 < nit) load(it + 2, u[0], h[0], cc1[0], cm1[0]);
      mma(u[1], h[1], cc1[1], cm1[1]);
    }
  }
  const int ac = a0 + m;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int b = NB * bp + j;
#pragma unroll
    for (int f = 0; f < FNO; ++f)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int l = 16 * f + kq + 4 * rr;
        if (l < no && ac < nv && b < nv)
          OtT[(((int64_t)p * no + l) * nvl + b) * nvl + ac] += acc[j][f][rr];
      }
  }
}

template <int FNO>
__global__ __launch_bounds__(256) void k_omega_oo(const double* __restrict__ cubes,
                                                  const double* __restrict__ Hs,
                                                  const int* __restrict__ tri, int ntri,
                                                  double* __restrict__ OtT, int no, int nv,
                                                  int tiles_a) {
  omega_oo_body<FNO>(cubes, Hs, tri, ntri, OtT, no, nv, tiles_a, blockIdx.x, blockIdx.y);
}

// For output block (p, x):
//   Ot2[p][x][a][d] += sum of Pvv[z][pi][chunk][a][d] over the batch's (triple,
//                      permutation) pairs with that p and q == x, and chunks;
//   Ot1[p][a]       += column nv of Pvv (block x == 0).
// Fixed summation order: triple, permutation, chunk.
__device__ __forceinline__ void reduce_body(const int* __restrict__ tri, int ntri,
                                            const double* __restrict__ Pvv,
                                            double* __restrict__ Ot1, double* __restrict__ Ot2,
                                            int no, int nv, int nchunks, int bx, int by, int bz) {
  __shared__ int lz[PLIST_MAX], lqr[PLIST_MAX], cz[MAX_BATCH + 1];
  int cnt;
  const int p = bz, x = by;
  cnt = pairs_with_p(tri, ntri, p, no, lz, lqr, cz);
  const int64_t nvl = nv, nv2 = nvl * nvl;
  const int NV1 = nv + 1;
  const int64_t pvs = (int64_t)nvl * NV1;  // one chunk slab
  const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
  const bool o2 = e < nv2;
  const bool o1 = (x == 0) && e < nv;  // Omega1 element a = e
  if (!o2 && !o1) return;
  const int a = (int)(e / nvl), d = (int)(e % nvl);
  const int n = cnt;
  if (o2) {
    double s2 = 0.0;
    bool any = false;  // uniform: a block (p, x) without pairs leaves Ot2 as it is
    for (int t = 0; t < n; ++t) {
      if (lqr[t] / no != x) continue;
      any = true;
      const double* pv = Pvv + (int64_t)lz[t] * nchunks * pvs + (int64_t)a * NV1 + d;
#pragma unroll 16
      for (int c = 0; c < nchunks; ++c) s2 += pv[c * pvs];
    }
    if (any) Ot2[((int64_t)p * no + x) * nv2 + e] += s2;
  }
  if (o1) {
    double s1 = 0.0;
    for (int t = 0; t < n; ++t) {
      const double* pv = Pvv + (int64_t)lz[t] * nchunks * pvs + (int64_t)e * NV1 + nv;
#pragma unroll 16
      for (int c = 0; c < nchunks; ++c) s1 += pv[c * pvs];
    }
    Ot1[(int64_t)p * nvl + e] += s1;
  }
}

__global__ __launch_bounds__(256) void k_reduce(const int* __restrict__ tri, int ntri,
                                                const double* __restrict__ Pvv,
                                                double* __restrict__ Ot1, double* __restrict__ Ot2,
                                                int no, int nv, int nchunks) {
  reduce_body(tri, ntri, Pvv, Ot1, Ot2, no, nv, nchunks, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------------------
// Preparation for the Jacobian transformations (Algorithm 2): for each distinct
// occupied permutation (p,q,r) of a triple, with U = tau~_{pqr},
//   Zv[a][b][p][d] -= sum_c    U[a,b,c] g_{qdrc}     (g_{qdrc} = Jo[q][r][d][c])
//   Zo[a][q][p][l] += sum_{bc} U[a,b,c] g_{lbrc}     (g_{lbrc} = Jo[l][r][b][c])
// ---------------------------------------------------------------------------

// Zv, output-stationary: one workgroup per (p, b, 128 x 128 tile of (a, d)) sums the
// batch's (triple, permutation) pairs with that p, in batch order, over c, and
// subtracts the result from Zv (read-modify-write; the batches run in order).
typedef TileCfg<4, 2, 2, 4, 16> ZvCfg;

__global__ __launch_bounds__(ZvCfg::NT) void k_zv(const double* __restrict__ cubes,
                                                  const double* __restrict__ Jo,
                                                  const int* __restrict__ tri, int ntri,
                                                  double* __restrict__ Zv, int no, int nv,
                                                  int tiles_m, int tiles_n) {
  typedef ZvCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  __shared__ int lz[PLIST_MAX], lqr[PLIST_MAX], cz[MAX_BATCH + 1];
  int cnt;
  const int p = blockIdx.y;
  const int tpp = tiles_m * tiles_n;
  const int b = blockIdx.x / tpp, tile = blockIdx.x % tpp;
  const int m0 = (tile / tiles_n) * T::BM, n0 = (tile % tiles_n) * T::BN;
  cnt = pairs_with_p(tri, ntri, p, no, lz, lqr, cz);
  const int n = cnt;
  if (n == 0) return;
  const int64_t nvl = nv, nv2 = nvl * nvl;
  const int cs = (nv + T::BK - 1) / T::BK;
  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    const int t = s / cs;
    k0 = (s % cs) * T::BK;
    const int zp = lz[t], z = zp / 6, pi = zp % 6;
    int slot, sbb, sm, sk;
    u_view(pi, nv, cube_pitch(nv), slot, sbb, sm, sk);
    A = make_opnd(cubes + ((int64_t)z * NSLOT + slot) * cube_slot(nv) + (int64_t)b * sbb, sm, sk,
                  nv, nv, sm == 1);
    B = make_opnd(Jo + (int64_t)lqr[t] * nv2, nv, 1, nv, nv, false);  // rows d, k = c
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>(n * cs, m0, n0, ops, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = m0 + acc_row<T>(wm, fm, lane, rr);
        const int d = n0 + acc_col<T>(wn, fn, lane);
        if (a < nv && d < nv) Zv[(((int64_t)a * nv + b) * no + p) * nv + d] -= acc[fm][fn][rr];
      }
}

// Zo partials: per (triple, permutation, 128-row tile of a, 16-column tile of l, b chunk)
//   Pzo[z][pi][chunk][a][l] = sum_{b in chunk} sum_c U[a,b,c] Jo[l][r][b][c]   (l < no)
// The l extent is no (12 at the benchmark size), so the tile is 128 x 16: eight
// wavefronts of 16 x 16, and the stage is mostly the streamed U rows.
typedef TileCfg<8, 1, 1, 1, 16> ZoCfg;

__global__ __launch_bounds__(ZoCfg::NT) void k_zo(const double* __restrict__ cubes,
                                                  const double* __restrict__ Jo,
                                                  const int* __restrict__ tri,
                                                  double* __restrict__ Pzo, int no, int nv,
                                                  int nbchunks) {
  typedef ZoCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  const int pi = blockIdx.y, z = blockIdx.z;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  if (!perm_active(tri_kind(i, j, k), pi)) return;
  int p, q, r;
  perm_pqr(pi, i, j, k, p, q, r);
  const int tm = (nv + T::BM - 1) / T::BM;
  const int bc = blockIdx.x % nbchunks;
  const int m0 = ((blockIdx.x / nbchunks) % tm) * T::BM;
  const int n0 = (blockIdx.x / nbchunks / tm) * T::BN;
  const int bb0 = (int)((int64_t)bc * nv / nbchunks);
  const int bb1 = (int)((int64_t)(bc + 1) * nv / nbchunks);
  if (bb0 >= bb1) return;
  const int64_t nvl = nv, nv2 = nvl * nvl;
  int slot, sbb, sm, sk;
  u_view(pi, nv, cube_pitch(nv), slot, sbb, sm, sk);
  const double* ub = cubes + ((int64_t)z * NSLOT + slot) * cube_slot(nv);
  const int cs = (nv + T::BK - 1) / T::BK;
  auto ops = [&](int s, Opnd& A, Opnd& B, int& k0) {
    const int b = bb0 + s / cs;
    k0 = (s % cs) * T::BK;
    A = make_opnd(ub + (int64_t)b * sbb, sm, sk, nv, nv, sm == 1);
    B = make_opnd(Jo + (int64_t)r * nv2 + (int64_t)b * nv, (int64_t)no * nv2, 1, no, nv, false);
  };
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  k_loop<T>((bb1 - bb0) * cs, m0, n0, ops, acc, lds);
  double* out = Pzo + (((int64_t)z * 6 + pi) * nbchunks + bc) * nvl * no;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = m0 + acc_row<T>(wm, fm, lane, rr);
        const int l = n0 + acc_col<T>(wn, fn, lane);
        if (a < nv && l < no) out[(int64_t)a * no + l] = acc[fm][fn][rr];
      }
}

// Zo[a][q][p][l] += the chunk sums of the batch's pairs with that (p, q), in batch order.
__global__ __launch_bounds__(256) void k_zo_reduce(const int* __restrict__ tri, int ntri,
                                                   const double* __restrict__ Pzo,
                                                   double* __restrict__ Zo, int no, int nv,
                                                   int nbchunks) {
  __shared__ int lz[PLIST_MAX], lqr[PLIST_MAX], cz[MAX_BATCH + 1];
  int cnt;
  const int q = blockIdx.y, p = blockIdx.z;
  cnt = pairs_with_p(tri, ntri, p, no, lz, lqr, cz);
  const int n = cnt;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0 || e >= (int64_t)nv * no) return;
  const int a = (int)(e / no), l = (int)(e % no);
  const int64_t slab = (int64_t)nv * no;
  double s = 0.0;
  for (int t = 0; t < n; ++t) {
    if (lqr[t] / no != q) continue;
    const double* pz = Pzo + (int64_t)lz[t] * nbchunks * slab + e;
    for (int c = 0; c < nbchunks; ++c) s += pz[c * slab];
  }
  Zo[(((int64_t)a * no + q) * no + p) * no + l] += s;
}

void launch_zv(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Zv, int no,
               int nv, hipStream_t st) {
  typedef ZvCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + T::BN - 1) / T::BN;
  hipLaunchKernelGGL(k_zv, dim3(nv * tm * tn, no), dim3(T::NT), 0, st, cubes, b.Jo, tri, ntri, Zv,
                     no, nv, tm, tn);
}

void launch_zo(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Pzo,
               double* Zo, int no, int nv, hipStream_t st, bool reduce) {
  typedef ZoCfg T;
  const int nbc = zo_nbchunks(nv, ntri);
  if (!reduce) {
    const int tm = (nv + T::BM - 1) / T::BM, tn = (no + T::BN - 1) / T::BN;
    hipLaunchKernelGGL(k_zo, dim3(nbc * tm * tn, 6, ntri), dim3(T::NT), 0, st, cubes, b.Jo, tri,
                       Pzo, no, nv, nbc);
  } else {
    hipLaunchKernelGGL(k_zo_reduce, dim3(nblk((int64_t)nv * no, 256), no, no), dim3(256), 0, st,
                       tri, ntri, Pzo, Zo, no, nv, nbc);
  }
}

double zprep_flops(int no, int nv, const int* kinds, int n) {
  const double v = nv, o = no;
  double perms = 0;
  for (int t = 0; t < n; ++t) perms += (kinds[t] == 0) ? 6 : 3;
  return perms * (2.0 * v * v * v * v + 2.0 * v * v * v * o);
}

// Split-K chunks of the b index of the Zo partials per (triple, permutation, a
// tile): about 2048 workgroups per launch, as a multiple of 8 beyond 8.
int zo_nbchunks(int nv, int ntri) {
  const int t = (nv + 127) / 128;
  const int per = 6 * t * t * (ntri > 0 ? ntri : 1);
  int nbc = (2048 + per - 1) / per;
  if (nbc > 8) nbc = (nbc + 7) / 8 * 8;
  if (nbc > nv) nbc = nv;
  return nbc < 1 ? 1 : nbc;
}

// K chunks (runs of whole LDS stages) of the Omega GEMM of one (triple,
// permutation, tile): enough workgroups for several rounds over the chip (two
// resident per CU), as a multiple of 8 beyond 8 so that the tiles of one
// (triple, permutation, chunk) -- which share operand rows -- are dispatched to
// the same XCD (workgroups go round-robin over the 8 XCDs in linear order, and
// tiles of one chunk are nchunks apart) and meet in its L2; at least 16 stages
// per chunk.
int omega_kchunks(int nv, int ntri, bool fp32acc) {
  static const int target = [] {
    const char* e = getenv("CC3_OMEGA_WG");
    const int v = e ? atoi(e) : 0;
    return v > 0 ? v : 2048;
  }();
  typedef OCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + 1 + T::BN - 1) / T::BN;
  const int per = 6 * tm * tn * (ntri > 0 ? ntri : 1);
  int nch = (target + per - 1) / per;
  if (nch > 8) nch = (nch + 7) / 8 * 8;
  const int S = (nv * nv + T::BK - 1) / T::BK;
  const int cap = S / 16 > 1 ? S / 16 : 1;
  if (nch > cap) nch = cap;
  // chunks that the MFMA sums in FP32 (the mixed-all forms) hold at most 4096 k, so
  // that their rounding does not grow with the batch (the split-BF16 form's K is the
  // blocked lp_kb_len(nv) >= nv^2)
  if (fp32acc) {
    const int need = (int)((lp_kb_len(nv) + 4095) / 4096);
    if (nch < need) nch = need > 8 ? (need + 7) / 8 * 8 : need;
  }
  return nch < 1 ? 1 : nch;
}

void launch_omega(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Pvv,
                  int no, int nv, hipStream_t st) {
  typedef OCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + 1 + T::BN - 1) / T::BN;
  const int nch = omega_kchunks(nv, ntri);
  hipLaunchKernelGGL(k_omega<double>, dim3(nch * tm * tn, 6, ntri), dim3(T::NT), 0, st, cubes,
                     (int)NSLOT, 0, b.Gbc, b.Gcb, tri, Pvv, no, nv, nch, tn);
}

void launch_omega_f32(const float* cubesF, const float* GbcF, const float* GcbF, const int* tri,
                      int ntri, double* Pvv, int no, int nv, hipStream_t st) {
  typedef OCfg T;
  const int tm = (nv + T::BM - 1) / T::BM, tn = (nv + 1 + T::BN - 1) / T::BN;
  const int nch = omega_kchunks(nv, ntri, true);
  hipLaunchKernelGGL(k_omega<float>, dim3(nch * tm * tn, 6, ntri), dim3(T::NT), 0, st, cubesF, 2,
                     (int)SLOT_TT, GbcF, GcbF, tri, Pvv, no, nv, nch, tn);
}

// FP32 copies for the mixed-all form: dst[e] = (float)src[e]
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

void launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  unsigned g = nblk(n, 256);
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_to_f32, dim3(g), dim3(256), 0, st, src, dst, n);
}

void launch_omega_oo(const double* cubes, const Blocks& b, const int* tri, int ntri, double* OtT,
                     int no, int nv, hipStream_t st) {
  const int ta = (nv + 63) / 64;
  const dim3 grid(((nv + 1) / 2) * ta, no), block(256);
  if (no <= 16)
    hipLaunchKernelGGL(k_omega_oo<1>, grid, block, 0, st, cubes, b.Hs, tri, ntri, OtT, no, nv, ta);
  else if (no <= 32)
    hipLaunchKernelGGL(k_omega_oo<2>, grid, block, 0, st, cubes, b.Hs, tri, ntri, OtT, no, nv, ta);
  else if (no <= 48)
    hipLaunchKernelGGL(k_omega_oo<3>, grid, block, 0, st, cubes, b.Hs, tri, ntri, OtT, no, nv, ta);
  else
    hipLaunchKernelGGL(k_omega_oo<4>, grid, block, 0, st, cubes, b.Hs, tri, ntri, OtT, no, nv, ta);
}

void launch_reduce(const int* tri, int ntri, const double* Pvv, double* Ot1, double* Ot2, int no,
                   int nv, bool fp32acc, hipStream_t st) {
  const int nch = omega_kchunks(nv, ntri, fp32acc);
  const int64_t nv2 = (int64_t)nv * nv;
  hipLaunchKernelGGL(k_reduce, dim3(nblk(nv2, 256), no, no), dim3(256), 0, st, tri, ntri, Pvv, Ot1,
                     Ot2, no, nv, nch);
}

// ---------------------------------------------------------------------------
// Packed persistent launches of the triple loop (serving): each workgroup takes
// work items blockIdx.x, blockIdx.x + gridDim.x, ... of the union of the jobs'
// unpacked grids and runs the same body on the job's operands, so each job's
// arithmetic is exactly that of its own launch.
// ---------------------------------------------------------------------------
__device__ inline int pack_job(const PackJob* __restrict__ jobs, int njobs, int kind,
                               unsigned item) {
  int r = 0;
  while (r + 1 < njobs && item >= jobs[r + 1].first[kind]) ++r;
  return r;
}

__global__ __launch_bounds__(WCfg::NT) void k_pack_wbuild(const PackJob* __restrict__ jobs,
                                                          int njobs, unsigned total) {
  typedef WCfg T;
  for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
    const PackJob& J = jobs[pack_job(jobs, njobs, PK_W, item)];
    const unsigned local = item - J.first[PK_W];
    const int tm = (J.nv + T::BM - 1) / T::BM, tn = (J.nv + T::BN - 1) / T::BN;
    const unsigned gx = (unsigned)J.nv * tm * tn;
    const int64_t cs = cube_slot(J.nv);
    wbuild_body<0>(J.t2, J.t2N, J.Gw, J.Go, J.tri, J.cubes, NSLOT * cs, cs, cube_pitch(J.nv), J.no,
                   J.nv, tm, tn, 0, (int)(local % gx), (int)((local / gx) % 3),
                   (int)(local / (gx * 3)));
    __syncthreads();
  }
}

__global__ __launch_bounds__(512) void k_pack_mix(const PackJob* __restrict__ jobs, int njobs,
                                                  unsigned total) {
  for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
    const PackJob& J = jobs[pack_job(jobs, njobs, PK_MIX, item)];
    const unsigned local = item - J.first[PK_MIX];
    const int nb = (J.nv + MT - 1) / MT;
    const unsigned nbt = (unsigned)(nb * (nb + 1) * (nb + 2) / 6);
    mix_body<512>(J.eps, J.tri, J.cubes, nullptr, nullptr, 0, J.no, J.nv, (int)(local % nbt),
                  (int)(local / nbt));
    __syncthreads();
  }
}

__global__ __launch_bounds__(OCfg::NT) void k_pack_omega(const PackJob* __restrict__ jobs,
                                                         int njobs, unsigned total) {
  typedef OCfg T;
  for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
    const PackJob& J = jobs[pack_job(jobs, njobs, PK_OMEGA, item)];
    const unsigned local = item - J.first[PK_OMEGA];
    const int tm = (J.nv + T::BM - 1) / T::BM, tn = (J.nv + 1 + T::BN - 1) / T::BN;
    const unsigned gx = (unsigned)J.nch * tm * tn;
    omega_body<double>(J.cubes, (int)NSLOT, 0, J.Gbc, J.Gcb, J.tri, J.Pvv, J.no, J.nv, J.nch, tn,
                       (int)(local % gx), (int)((local / gx) % 6), (int)(local / (gx * 6)));
    __syncthreads();
  }
}

template <int FNO>
__global__ __launch_bounds__(256) void k_pack_omega_oo(const PackJob* __restrict__ jobs, int njobs,
                                                       unsigned total) {
  for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
    const PackJob& J = jobs[pack_job(jobs, njobs, PK_OO, item)];
    const unsigned local = item - J.first[PK_OO];
    const int ta = (J.nv + 63) / 64;
    const unsigned gx = (unsigned)((J.nv + 1) / 2) * ta;
    omega_oo_body<FNO>(J.cubes, J.Hs, J.tri, J.ntri, J.OtT, J.no, J.nv, ta, (int)(local % gx),
                       (int)(local / gx));
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_pack_reduce(const PackJob* __restrict__ jobs, int njobs,
                                                     unsigned total) {
  for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
    const PackJob& J = jobs[pack_job(jobs, njobs, PK_RED, item)];
    const unsigned local = item - J.first[PK_RED];
    const unsigned gx = (unsigned)(((int64_t)J.nv * J.nv + 255) / 256);
    reduce_body(J.tri, J.ntri, J.Pvv, J.Ot1, J.Ot2, J.no, J.nv, J.nch, (int)(local % gx),
                (int)((local / gx) % J.no), (int)(local / (gx * J.no)));
    __syncthreads();
  }
}

void pack_items(const PackJob& j, unsigned (&items)[PK_N]) {
  const int no = j.no, nv = j.nv, nt = j.ntri;
  const unsigned tw = (unsigned)((nv + WCfg::BM - 1) / WCfg::BM) * ((nv + WCfg::BN - 1) / WCfg::BN);
  items[PK_W] = (unsigned)nv * tw * 3u * nt;
  const int nb = (nv + MT - 1) / MT;
  items[PK_MIX] = (unsigned)(nb * (nb + 1) * (nb + 2) / 6) * nt;
  const unsigned to = (unsigned)((nv + OCfg::BM - 1) / OCfg::BM) * ((nv + 1 + OCfg::BN - 1) / OCfg::BN);
  items[PK_OMEGA] = (unsigned)j.nch * to * 6u * nt;
  items[PK_OO] = (unsigned)((nv + 1) / 2) * ((nv + 63) / 64) * no;
  items[PK_RED] = nblk((int64_t)nv * nv, 256) * no * no;
}

// persistent grids: a few rounds of resident workgroups, never more than the items
static unsigned pack_grid(unsigned total, unsigned cap) { return total < cap ? total : cap; }

void launch_wbuild_lp_packed(const PackJob* jobs, int njobs, unsigned total, int prec,
                             hipStream_t st);

void launch_packed_step(const PackJob* dev_jobs, const PackJob* host_jobs, int njobs, int prec,
                        hipStream_t st) {
  if (njobs <= 0) return;
  unsigned total[PK_N] = {0, 0, 0, 0, 0};
  int max_no = 1;
  for (int r = 0; r < njobs; ++r) {
    unsigned it[PK_N];
    pack_items(host_jobs[r], it);
    for (int k = 0; k < PK_N; ++k) total[k] += it[k];
    max_no = std::max(max_no, host_jobs[r].no);
  }
  if (prec == CC3_FP64)
    hipLaunchKernelGGL(k_pack_wbuild, dim3(pack_grid(total[PK_W], 2048)), dim3(WCfg::NT), 0, st,
                       dev_jobs, njobs, total[PK_W]);
  else
    launch_wbuild_lp_packed(dev_jobs, njobs, total[PK_W], prec, st);
  hipLaunchKernelGGL(k_pack_mix, dim3(pack_grid(total[PK_MIX], 4096)), dim3(512), 0, st, dev_jobs,
                     njobs, total[PK_MIX]);
  hipLaunchKernelGGL(k_pack_omega, dim3(pack_grid(total[PK_OMEGA], 2048)), dim3(OCfg::NT), 0, st,
                     dev_jobs, njobs, total[PK_OMEGA]);
  const dim3 goo(pack_grid(total[PK_OO], 8192));
  if (max_no <= 16)
    hipLaunchKernelGGL(k_pack_omega_oo<1>, goo, dim3(256), 0, st, dev_jobs, njobs, total[PK_OO]);
  else if (max_no <= 32)
    hipLaunchKernelGGL(k_pack_omega_oo<2>, goo, dim3(256), 0, st, dev_jobs, njobs, total[PK_OO]);
  else if (max_no <= 48)
    hipLaunchKernelGGL(k_pack_omega_oo<3>, goo, dim3(256), 0, st, dev_jobs, njobs, total[PK_OO]);
  else
    hipLaunchKernelGGL(k_pack_omega_oo<4>, goo, dim3(256), 0, st, dev_jobs, njobs, total[PK_OO]);
  hipLaunchKernelGGL(k_pack_reduce, dim3(pack_grid(total[PK_RED], 16384)), dim3(256), 0, st,
                     dev_jobs, njobs, total[PK_RED]);
}

// FLOP of the dominant contractions and their companions, padding excluded.
double wbuild_flops(int no, int nv, const int* kinds, int n) {
  const double v = nv, o = no;
  const double term = 2.0 * v * v * v * v + 2.0 * v * v * v * o;
  double f = 0.0;
  for (int t = 0; t < n; ++t) f += (kinds[t] == TRI_DISTINCT ? 6.0 : 3.0) * term;
  return f;
}

// k_omega: the vv term (2 nv^4) and Omega1 (2 nv^3) per permutation
double omega_flops(int no, int nv, const int* kinds, int n) {
  const double v = nv;
  const double perm = 2.0 * v * v * v * v + 2.0 * v * v * v;
  double f = 0.0;
  for (int t = 0; t < n; ++t) f += (kinds[t] == TRI_DISTINCT ? 6.0 : 3.0) * perm;
  (void)no;
  return f;
}

// k_omega_oo: the oo and Fock terms (2 nv^3 no) per permutation
double omega_oo_flops(int no, int nv, const int* kinds, int n) {
  const double v = nv, o = no;
  double f = 0.0;
  for (int t = 0; t < n; ++t) f += (kinds[t] == TRI_DISTINCT ? 6.0 : 3.0) * 2.0 * v * v * v * o;
  return f;
}

}  // namespace cc3
