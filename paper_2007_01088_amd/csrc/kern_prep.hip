// Preparation kernels run once per residual call, before the triple loop:
// the T1 transformation of the Cholesky vectors, the Fock ov block, the
// integral-block build (FP64 MFMA GEMMs over the Cholesky index, writing the
// internal layouts the triple loop streams), the re-layout of caller-given
// blocks, the triple table, and the covariant back-transformation after it.
#include "cc3_device.hpp"
#include "cc3_internal.hpp"

namespace cc3 {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = nblk(n, 256);
  if (g > 65536u) g = 65536u;
  hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, st, p, n, v);
}

__global__ void k_add(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) y[i] += x[i];
}

void launch_add(double* y, const double* x, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = nblk(n, 256);
  if (g > 65536u) g = 65536u;
  hipLaunchKernelGGL(k_add, dim3(g), dim3(256), 0, st, y, x, n);
}

// ---------------------------------------------------------------------------
// T1 transformation (exp(-T1) H exp(T1)):  Lt = (1 - t) L (1 + t), t[no+a][i] = t1[i][a].
//   Lt_bd = L_bd - sum_l t1[l][b] L_ld        Lt_lj = L_lj + sum_d L_ld t1[j][d]
//   Lt_ck = L_ck + sum_d L_cd t1[k][d] - sum_l t1[l][c] Lt_lk      Lt_kc = L_kc
// ---------------------------------------------------------------------------
__global__ void k_t1_vv(const double* __restrict__ L, const double* __restrict__ t1,
                        double* __restrict__ Lvv, int no, int nv) {
  const int J = blockIdx.y;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nv * nv) return;
  const int b = (int)(idx / nv), d = (int)(idx % nv);
  const int nmo = no + nv;
  const double* LJ = L + (int64_t)J * nmo * nmo;
  double v = LJ[(int64_t)(no + b) * nmo + no + d];
  for (int l = 0; l < no; ++l) v -= t1[(int64_t)l * nv + b] * LJ[(int64_t)l * nmo + no + d];
  const int64_t base = (int64_t)J * nv * nv;
  Lvv[base + (int64_t)b * nv + d] = v;
}

__global__ void k_t1_oo(const double* __restrict__ L, const double* __restrict__ t1,
                        double* __restrict__ Loo, double* __restrict__ LooT,
                        double* __restrict__ Lov, int no, int nv) {
  const int J = blockIdx.y;
  const int nmo = no + nv;
  const double* LJ = L + (int64_t)J * nmo * nmo;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < no * no) {
    const int l = idx / no, j = idx % no;
    double v = LJ[(int64_t)l * nmo + j];
    for (int d = 0; d < nv; ++d) v += LJ[(int64_t)l * nmo + no + d] * t1[(int64_t)j * nv + d];
    Loo[(int64_t)J * no * no + (int64_t)l * no + j] = v;
    LooT[(int64_t)J * no * no + (int64_t)j * no + l] = v;
  }
  // untransformed ov block, Lov[J][k][c] = L_{k, no+c}
  for (int e = idx; e < no * nv; e += gridDim.x * blockDim.x) {
    const int k = e / nv, c = e % nv;
    Lov[(int64_t)J * no * nv + e] = LJ[(int64_t)k * nmo + no + c];
  }
}

// LvoT[J][k][c] for 16 consecutive c of one J.  The rows L_{no+c, no+d} and t1
// pass through LDS in chunks of 64 d, so every global read is a row segment;
// each sum keeps the order of the formula above (d ascending, then l).
__global__ __launch_bounds__(256) void k_t1_vo(const double* __restrict__ L,
                                               const double* __restrict__ t1,
                                               const double* __restrict__ Loo,
                                               double* __restrict__ LvoT, int no, int nv) {
  constexpr int RC = 16, DC = 64, PER = (RC * 64 + 255) / 256;  // no <= 63
  __shared__ double Ls[RC][DC + 1];
  __shared__ double Ts[64][DC + 1];
  const int J = blockIdx.y, c0 = blockIdx.x * RC, tid = threadIdx.x;
  const int nmo = no + nv;
  const double* LJ = L + (int64_t)J * nmo * nmo;
  double acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + 256 * i, ci = e % RC, k = e / RC, c = c0 + ci;
    acc[i] = (k < no && c < nv) ? LJ[(int64_t)(no + c) * nmo + k] : 0.0;
  }
  for (int d0 = 0; d0 < nv; d0 += DC) {
    const int dn = min(DC, nv - d0);
    for (int e = tid; e < RC * DC; e += 256) {
      const int ci = e / DC, dd = e % DC, c = c0 + ci;
      Ls[ci][dd] = (c < nv && dd < dn) ? LJ[(int64_t)(no + c) * nmo + no + d0 + dd] : 0.0;
    }
    for (int e = tid; e < no * DC; e += 256) {
      const int k = e / DC, dd = e % DC;
      Ts[k][dd] = dd < dn ? t1[(int64_t)k * nv + d0 + dd] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + 256 * i, ci = e % RC, k = e / RC;
      if (k < no) {
        double v = acc[i];
        for (int dd = 0; dd < dn; ++dd) v += Ls[ci][dd] * Ts[k][dd];
        acc[i] = v;
      }
    }
    __syncthreads();
  }
  const double* LooJ = Loo + (int64_t)J * no * no;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + 256 * i, ci = e % RC, k = e / RC, c = c0 + ci;
    if (k >= no || c >= nv) continue;
    double v = acc[i];
    for (int l = 0; l < no; ++l) v -= t1[(int64_t)l * nv + c] * LooJ[(int64_t)l * no + k];
    LvoT[(int64_t)J * no * nv + (int64_t)k * nv + c] = v;
  }
}

void launch_t1_transform(const double* L, const double* t1, const CholeskyScratch& cs, int no,
                         int nv, int nJ, hipStream_t st) {
  hipLaunchKernelGGL(k_t1_vv, dim3(nblk((int64_t)nv * nv, 256), nJ), dim3(256), 0, st, L, t1,
                     cs.Lvv, no, nv);
  int m = no * no > no * nv ? no * no : no * nv;
  hipLaunchKernelGGL(k_t1_oo, dim3(nblk(m, 256), nJ), dim3(256), 0, st, L, t1, cs.Loo, cs.LooT,
                     cs.Lov, no, nv);
  hipLaunchKernelGGL(k_t1_vo, dim3(nblk(nv, 16), nJ), dim3(256), 0, st, L, t1, cs.Loo, cs.LvoT,
                     no, nv);
}

// ---------------------------------------------------------------------------
// Fock ov block of the T1-transformed Hamiltonian (canonical reference):
//   F_kc = sum_ld t1[l][d] (2 g_kcld - g_kdlc),  g_kcld = sum_J L_kc L_ld
//        = sum_J [ 2 s_J L_kc - sum_l M_J[k][l] L_lc ],
//   s_J = sum_ld t1[l][d] L_ld,  M_J[k][l] = sum_d L_kd t1[l][d].
// ---------------------------------------------------------------------------
__global__ void k_fock_sm(const double* __restrict__ t1, const double* __restrict__ Lov,
                          double* __restrict__ s, double* __restrict__ M, int no, int nv) {
  const int J = blockIdx.x;
  const double* LJ = Lov + (int64_t)J * no * nv;
  __shared__ double red[256];
  double acc = 0.0;
  for (int e = threadIdx.x; e < no * nv; e += blockDim.x) acc += t1[e] * LJ[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) s[J] = red[0];
  for (int e = threadIdx.x; e < no * no; e += blockDim.x) {
    const int k = e / no, l = e % no;
    double v = 0.0;
    for (int d = 0; d < nv; ++d) v += LJ[(int64_t)k * nv + d] * t1[(int64_t)l * nv + d];
    M[(int64_t)J * no * no + e] = v;
  }
}

// F[k][c] for 64 consecutive c of one k; sixteen slices of the Cholesky index
// summed through LDS in a fixed order.
__global__ __launch_bounds__(1024) void k_fock(const double* __restrict__ Lov,
                                               const double* __restrict__ s,
                                               const double* __restrict__ M, double* __restrict__ F,
                                               int no, int nv, int nJ) {
  constexpr int NS = 16;
  __shared__ double red[64 * NS];
  const int k = blockIdx.x;
  const int c = blockIdx.y * 64 + (threadIdx.x & 63);
  const int js = threadIdx.x >> 6;
  double v = 0.0;
  if (c < nv) {
    for (int J = js; J < nJ; J += NS) {
      const double* LJ = Lov + (int64_t)J * no * nv;
      double w = 2.0 * s[J] * LJ[(int64_t)k * nv + c];
      const double* MJ = M + (int64_t)J * no * no + (int64_t)k * no;
      for (int l = 0; l < no; ++l) w -= MJ[l] * LJ[(int64_t)l * nv + c];
      v += w;
    }
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = NS / 2; h >= 1; h >>= 1) {
    if (js < h) red[threadIdx.x] += red[threadIdx.x + 64 * h];
    __syncthreads();
  }
  if (js == 0 && c < nv) F[(int64_t)k * nv + c] = red[threadIdx.x];
}

void launch_fock(const double* t1, const CholeskyScratch& cs, double* F, int no, int nv, int nJ,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_fock_sm, dim3(nJ), dim3(256), 0, st, t1, cs.Lov, cs.s, cs.M, no, nv);
  hipLaunchKernelGGL(k_fock, dim3(no, nblk(nv, 64)), dim3(1024), 0, st, cs.Lov, cs.s, cs.M, F, no,
                     nv, nJ);
}

// ---------------------------------------------------------------------------
// Integral-block build: C[m][n] = sum_J A(m, J) B(J, n) on FP64 MFMA, batched
// over blockIdx.z, with an output map per block kind.
// ---------------------------------------------------------------------------
enum BuildKind { BUILD_PLAIN = 0, BUILD_JO = 1, BUILD_HS = 2, BUILD_GO = 3, BUILD_GW = 4 };

typedef TileCfg<4, 2, 2, 4, 16> BuildCfg;  // 8 wavefronts, 128 x 128 tiles

// One product of a grouped build launch: C_z = A_z B_z for z < batch, with
// A(m, J) at A[z * a_bs + m * a_sm + J * a_sk], B(J, n) at B[z * b_bs + J * b_sk + n * b_sn].
struct BuildProb {
  const double* A;
  const double* B;
  double* C;
  int64_t a_sm, a_sk, a_bs, b_sk, b_sn, b_bs, c_bs;
  int M, N, kind, batch;
};
enum { MAX_BUILD_PROBS = 6 };
// The products of one launch, all with the same K; workgroups first0[p] ..
// first0[p + 1] - 1 take the tiles of product p.
struct BuildSet {
  BuildProb p[MAX_BUILD_PROBS];
  unsigned first0[MAX_BUILD_PROBS + 1];
  int n, K, no, nv;
  const double* F;
};

__global__ __launch_bounds__(BuildCfg::NT, 2) void k_build(const BuildSet set) {
  typedef BuildCfg T;
  __shared__ double lds[T::LDS_DOUBLES];
  int pi = 0;
  while (pi + 1 < set.n && blockIdx.x >= set.first0[pi + 1]) ++pi;
  const BuildProb& pr = set.p[pi];
  const int M = pr.M, N = pr.N, K = set.K, kind = pr.kind, no = set.no, nv = set.nv;
  const int mt = (M + T::BM - 1) / T::BM, nt = (N + T::BN - 1) / T::BN;
  const unsigned local = blockIdx.x - set.first0[pi];
  const int z = (int)(local / (unsigned)(mt * nt));
  const int t = (int)(local % (unsigned)(mt * nt));
  const int m0 = (t % mt) * T::BM;
  const int n0 = (t / mt) * T::BN;
  const double* A = pr.A + (int64_t)z * pr.a_bs;
  const double* B = pr.B + (int64_t)z * pr.b_bs;
  d4v acc[T::FM][T::FN];
  zero_acc<T>(acc);
  const int nsteps = (K + T::BK - 1) / T::BK;
  auto ops = [&](int s, Opnd& oa, Opnd& ob, int& k0) {
    k0 = s * T::BK;
    oa = make_opnd(A, pr.a_sm, pr.a_sk, M, K, true);
    ob = make_opnd(B, pr.b_sn, pr.b_sk, N, K, true);
  };
  k_loop<T>(nsteps, m0, n0, ops, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double* Cz = pr.C + (int64_t)z * pr.c_bs;
  const double* F = set.F;
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + acc_row<T>(wm, fm, lane, r);
        const int n = n0 + acc_col<T>(wn, fn, lane);
        if (m >= M || n >= N) continue;
        const double v = acc[fm][fn][r];
        if (kind == BUILD_PLAIN) {
          Cz[(int64_t)m * N + n] = v;
        } else if (kind == BUILD_JO) {  // m = q*nv + b, n = r*nv + c -> Jo[q][r][b][c]
          const int q = m / nv, b = m % nv, rr = n / nv, c = n % nv;
          Cz[(((int64_t)q * no + rr) * nv + b) * nv + c] = v;
        } else if (kind == BUILD_HS) {  // m = q*no + l, n = r*nv + c -> Hs[q][r][c][l]
          const int q = m / no, l = m % no, rr = n / nv, c = n % nv;
          Cz[(((int64_t)q * no + rr) * nv + c) * no + l] = (l == q ? F[(int64_t)rr * nv + c] : 0.0) - v;
        } else if (kind == BUILD_GO) {  // m = q*no + l, n = r*nv + z -> Go[q][r][z][l]
          const int q = m / no, l = m % no, rr = n / nv, c = n % nv;
          Cz[(((int64_t)q * no + rr) * nv + c) * no + l] = v;
        } else {  // BUILD_GW: m = z, n = y*nv + d -> Gw[r][y][z][d] (batch r)
          const int y = n / nv, d = n % nv;
          Cz[((int64_t)y * nv + m) * nv + d] = v;
        }
      }
}

static void add_build(BuildSet& set, const double* A, int64_t a_sm, int64_t a_sk, int64_t a_bs,
                      const double* B, int64_t b_sk, int64_t b_sn, int64_t b_bs, int M, int N,
                      double* C, int64_t c_bs, int batch, int kind) {
  BuildProb& p = set.p[set.n++];
  p.A = A; p.a_sm = a_sm; p.a_sk = a_sk; p.a_bs = a_bs;
  p.B = B; p.b_sk = b_sk; p.b_sn = b_sn; p.b_bs = b_bs;
  p.C = C; p.c_bs = c_bs;
  p.M = M; p.N = N; p.kind = kind; p.batch = batch;
}

static void launch_build_set(BuildSet& set, hipStream_t st) {
  typedef BuildCfg T;
  set.first0[0] = 0;
  for (int i = 0; i < set.n; ++i) {
    const BuildProb& p = set.p[i];
    set.first0[i + 1] = set.first0[i] + nblk(p.M, T::BM) * nblk(p.N, T::BN) * (unsigned)p.batch;
  }
  hipLaunchKernelGGL(k_build, dim3(set.first0[set.n]), dim3(T::NT), 0, st, set);
}

// Gcb[r][n][c][b] = Gbc[r][n][b][c]: nv x nv transposes, one per (r, n), through
// padded 32 x 32 LDS tiles.
__global__ __launch_bounds__(256) void k_gcb(const double* __restrict__ Gbc,
                                             double* __restrict__ Gcb, int nv) {
  __shared__ double t[32][33];
  const int tn = (nv + 31) / 32;
  const int64_t slab = blockIdx.x / (tn * tn);  // r * (nv + no) + n
  const int tile = blockIdx.x % (tn * tn);
  const int b0 = (tile / tn) * 32, c0 = (tile % tn) * 32;
  const int64_t nv2 = (int64_t)nv * nv;
  const double* src = Gbc + slab * nv2;
  double* dst = Gcb + slab * nv2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int b = b0 + y, c = c0 + tx;
    if (b < nv && c < nv) t[y][tx] = src[(int64_t)b * nv + c];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int c = c0 + y, b = b0 + tx;
    if (b < nv && c < nv) dst[(int64_t)c * nv + b] = t[tx][y];
  }
}

void launch_gcb(const Blocks& bl, int no, int nv, hipStream_t st) {
  const unsigned t = nblk(nv, 32);
  hipLaunchKernelGGL(k_gcb, dim3(t * t * no * (nv + no)), dim3(256), 0, st, bl.Gbc, bl.Gcb, nv);
}

void launch_build_blocks(const CholeskyScratch& cs, const Blocks& bl, int no, int nv, int nJ,
                         hipStream_t st) {
  const int64_t nv2 = (int64_t)nv * nv, nv3 = nv2 * nv, onv = (int64_t)no * nv;
  const int64_t gs = (int64_t)(nv + no) * nv2;  // one r slab of Gbc / Gcb
  // all six products share K = nJ: one launch, the large ones first
  BuildSet set = {};
  set.K = nJ; set.no = no; set.nv = nv; set.F = bl.F;
  // Gw[r][y][z][d] = sum_J LvoT[J][r][z] Lvv[J][(y,d)]   (rows z, columns (y,d), batch r)
  add_build(set, cs.LvoT, 1, onv, nv, cs.Lvv, nv2, 1, 0, nv, (int)nv2, bl.Gw, nv3, no, BUILD_GW);
  // Gbc[r][(d,b)][c] = sum_J Lvv[J][(d,b)] Lov[J][r][c]            (rows n = d < nv)
  add_build(set, cs.Lvv, 1, nv2, 0, cs.Lov, onv, 1, nv, (int)nv2, nv, bl.Gbc, gs, no, BUILD_PLAIN);
  // Gbc[r][nv + (l,b)][c] = sum_J Lov[J][(l,b)] Lov[J][r][c]      (rows n = nv + l)
  add_build(set, cs.Lov, 1, onv, 0, cs.Lov, onv, 1, nv, (int)onv, nv, bl.Gbc + nv3, gs, no,
            BUILD_PLAIN);
  // Jo[q][r][b][c] = sum_J Lov[J][q][b] Lov[J][r][c]
  add_build(set, cs.Lov, 1, onv, 0, cs.Lov, onv, 1, 0, (int)onv, (int)onv, bl.Jo, 0, 1, BUILD_JO);
  // Hs[q][r][c][l] = delta_lq F[r][c] - sum_J Loo[J][q][l] Lov[J][r][c]
  add_build(set, cs.Loo, 1, (int64_t)no * no, 0, cs.Lov, onv, 1, 0, no * no, (int)onv, bl.Hs, 0,
            1, BUILD_HS);
  // Go[q][r][z][l] = sum_J LooT[J][q][l] LvoT[J][r][z]   (LooT[J][q][l] = Lt_lq)
  add_build(set, cs.LooT, 1, (int64_t)no * no, 0, cs.LvoT, onv, 1, 0, no * no, (int)onv, bl.Go, 0,
            1, BUILD_GO);
  launch_build_set(set, st);
  launch_gcb(bl, no, nv, st);
}

// The blocks of the transition-density loop (Algorithm 3), in one grouped launch:
// Gw, Go and Jo as for the residual; Go3[p][q][z][l] = g_{plqz} = sum_J Lt_pl L_qz;
// Gl[p][y][z][d] = g_{pydz} = sum_J L_py Lt_dz, built as [p][y][d][z] into `tmp`
// (no nv^3 doubles) and transposed per (p, y) slab.
void launch_build_density_blocks(const CholeskyScratch& cs, double* Gw, double* Go, double* Jo,
                                 double* Go3, double* Gl, double* tmp, int no, int nv, int nJ,
                                 hipStream_t st) {
  const int64_t nv2 = (int64_t)nv * nv, nv3 = nv2 * nv, onv = (int64_t)no * nv;
  BuildSet set = {};
  set.K = nJ; set.no = no; set.nv = nv; set.F = nullptr;
  add_build(set, cs.LvoT, 1, onv, nv, cs.Lvv, nv2, 1, 0, nv, (int)nv2, Gw, nv3, no, BUILD_GW);
  // tmp[(p,y)][(d,z)] = sum_J Lov[J][p][y] Lvv[J][d][z]
  add_build(set, cs.Lov, 1, onv, 0, cs.Lvv, nv2, 1, 0, (int)onv, (int)nv2, tmp, 0, 1, BUILD_PLAIN);
  add_build(set, cs.Lov, 1, onv, 0, cs.Lov, onv, 1, 0, (int)onv, (int)onv, Jo, 0, 1, BUILD_JO);
  add_build(set, cs.LooT, 1, (int64_t)no * no, 0, cs.LvoT, onv, 1, 0, no * no, (int)onv, Go, 0,
            1, BUILD_GO);
  // Go3: m = p*no + l (Loo[J][p][l] = Lt_pl), n = q*nv + z (Lov[J][q][z] = L_qz)
  add_build(set, cs.Loo, 1, (int64_t)no * no, 0, cs.Lov, onv, 1, 0, no * no, (int)onv, Go3, 0, 1,
            BUILD_GO);
  launch_build_set(set, st);
  const unsigned t = nblk(nv, 32);
  hipLaunchKernelGGL(k_gcb, dim3(t * t * no * nv), dim3(256), 0, st, tmp, Gl, nv);
}

// ---------------------------------------------------------------------------
// Integral blocks given in the paper's index order -> internal layouts.
// ---------------------------------------------------------------------------
__global__ void k_relayout_vv(const double* __restrict__ g_vvvo_y, const double* __restrict__ g_vvov_y,
                              double* __restrict__ Gw, double* __restrict__ Gbc, int no, int nv,
                              int y0, int ny) {
  // output index (r, y, d, z) of an nv^3 slab, z fastest, for y in [y0, y0 + ny);
  // the inputs start at first index y0
  const int64_t nv2 = (int64_t)nv * nv, nv3 = nv2 * nv;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= (int64_t)ny * nv2) return;
  const int yl = (int)(e / nv2), d = (int)((e / nv) % nv), z = (int)(e % nv);
  const int64_t out = (int64_t)y0 * nv2 + e;
  // Gw[r][y][u][w] = g_vvvo[y][w][u][r]  (u = d, w = z: the contracted index w fastest)
  Gw[(int64_t)r * nv3 + out] = g_vvvo_y[(((int64_t)yl * nv + z) * nv + d) * no + r];
  // Gbc[r][n=y][b=d][c=z] = g_vvov[n][b][r][c]
  Gbc[(int64_t)r * (nv + no) * nv2 + out] = g_vvov_y[(((int64_t)yl * nv + d) * no + r) * nv + z];
}

__global__ void k_relayout_small(const double* __restrict__ g_oovo, const double* __restrict__ g_ovov,
                                 const double* __restrict__ g_ooov, const double* __restrict__ F_ov,
                                 double* __restrict__ Go, double* __restrict__ Jo,
                                 double* __restrict__ Gbc, double* __restrict__ Hs,
                                 double* __restrict__ F, int no, int nv) {
  const int q = blockIdx.y / no, r = blockIdx.y % no;
  const int64_t nv2 = (int64_t)nv * nv;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nv * nv; e += gridDim.x * blockDim.x) {
    const int b = e / nv, c = e % nv;  // Jo[q][r][b][c] = Gbc[r][nv + q][b][c] = g_ovov[q][b][r][c]
    const double g = g_ovov[(((int64_t)q * nv + b) * no + r) * nv + c];
    Jo[((int64_t)q * no + r) * nv2 + e] = g;
    Gbc[((int64_t)r * (nv + no) + nv + q) * nv2 + e] = g;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < no * nv; e += gridDim.x * blockDim.x) {
    const int l = e / nv, c = e % nv;
    // Go[q][r][z][l] = g_oovo[l][q][z][r]
    Go[(((int64_t)q * no + r) * nv + c) * no + l] = g_oovo[(((int64_t)l * no + q) * nv + c) * no + r];
    // Hs[q][r][c][l] = delta_lq F[r][c] - g_ooov[q][l][r][c]
    Hs[(((int64_t)q * no + r) * nv + c) * no + l] =
        (l == q ? F_ov[(int64_t)r * nv + c] : 0.0) - g_ooov[(((int64_t)q * no + l) * no + r) * nv + c];
  }
  if (blockIdx.y == 0)
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < no * nv; e += gridDim.x * blockDim.x)
      F[e] = F_ov[e];
}

void launch_relayout_small(const double* g_oovo, const double* g_ovov, const double* g_ooov,
                           const double* F_ov, const Blocks& b, int no, int nv, hipStream_t st) {
  unsigned gx = nblk((int64_t)nv * nv, 256);
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_relayout_small, dim3(gx, no * no), dim3(256), 0, st, g_oovo, g_ovov,
                     g_ooov, F_ov, b.Go, b.Jo, b.Gbc, b.Hs, b.F, no, nv);
}

void launch_relayout_vv(const double* g_vvvo_y, const double* g_vvov_y, int y0, int ny,
                        const Blocks& b, int no, int nv, hipStream_t st) {
  const int64_t n = (int64_t)ny * nv * nv;
  hipLaunchKernelGGL(k_relayout_vv, dim3(nblk(n, 256), no), dim3(256), 0, st, g_vvvo_y, g_vvov_y,
                     b.Gw, b.Gbc, no, nv, y0, ny);
}

// ---------------------------------------------------------------------------
// Triple table: the restricted loop i >= j >= k without the i == j == k triples,
// lexicographic rank L = C(i+2,3) + j(j+1)/2 + k - i, dealt round-robin over the
// nbatch batches: position = start of group L mod nbatch + L / nbatch.  Each
// batch then samples the whole loop, so that the (triple, permutation) pairs of
// a batch spread evenly over the first occupied index, which the
// output-stationary kernels are parallel over.
// ---------------------------------------------------------------------------
__global__ void k_triples(int* __restrict__ tri, int no, int nbatch) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= no * no * no) return;
  const int i = e / (no * no), j = (e / no) % no, k = e % no;
  if (!(i >= j && j >= k) || (i == j && j == k)) return;
  const int n = no * (no + 1) * (no + 2) / 6 - no;
  const int L = i * (i + 1) * (i + 2) / 6 + j * (j + 1) / 2 + k - i;
  const int g = L % nbatch;
  const int pos = g * (n / nbatch) + min(g, n % nbatch) + L / nbatch;
  tri[3 * pos + 0] = i;
  tri[3 * pos + 1] = j;
  tri[3 * pos + 2] = k;
}

void launch_triple_table(int* tri, int no, int nbatch, hipStream_t st) {
  hipLaunchKernelGGL(k_triples, dim3(nblk((int64_t)no * no * no, 256)), dim3(256), 0, st, tri, no,
                     nbatch < 1 ? 1 : nbatch);
}

void launch_set_triples(int* tri_dev, const int* host_tri, int n, hipStream_t st) {
  hipMemcpyAsync(tri_dev, host_tri, sizeof(int) * 3 * (size_t)n, hipMemcpyHostToDevice, st);
}

// ---------------------------------------------------------------------------
// Covariant back-transformation.  The contravariant doubles residual is held
// in two parts, Ot~[i][j][a][b] = Ot2[i][j][a][b] + OtT[i][j][b][a]; then
//   Omega^a_i = Ot^a_i
//   Omega^{ab}_{ij} = 1/3 [(2 Ot~^{ab}_{ij} + Ot~^{ba}_{ij}) + (2 Ot~^{ba}_{ji} + Ot~^{ab}_{ji})]
// ---------------------------------------------------------------------------
__device__ inline double ot2(const double* __restrict__ Ot2, const double* __restrict__ OtT,
                             int64_t ij, int64_t nv, int a, int b) {
  return Ot2[(ij + a) * nv + b] + OtT[(ij + b) * nv + a];
}

__global__ void k_back(const double* __restrict__ Ot1, const double* __restrict__ Ot2,
                       const double* __restrict__ OtT, double* __restrict__ O1,
                       double* __restrict__ O2, int no, int nv, int acc) {
  const int64_t nvl = nv, n2 = (int64_t)no * no * nvl * nvl;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n2) {
    const int b = (int)(e % nvl), a = (int)((e / nvl) % nvl);
    const int j = (int)((e / (nvl * nvl)) % no), i = (int)(e / (nvl * nvl * no));
    const int64_t ij = ((int64_t)i * no + j) * nvl, ji = ((int64_t)j * no + i) * nvl;
    const double v = (2.0 * ot2(Ot2, OtT, ij, nvl, a, b) + ot2(Ot2, OtT, ij, nvl, b, a) +
                      2.0 * ot2(Ot2, OtT, ji, nvl, b, a) + ot2(Ot2, OtT, ji, nvl, a, b)) / 3.0;
    O2[e] = acc ? O2[e] + v : v;
  }
  if (e < (int64_t)no * nv) O1[e] = acc ? O1[e] + Ot1[e] : Ot1[e];
}

void launch_back_transform(const double* Ot1, const double* Ot2, const double* OtT, double* O1,
                           double* O2, int no, int nv, bool accumulate, hipStream_t st) {
  const int64_t n2 = (int64_t)no * no * nv * nv;
  hipLaunchKernelGGL(k_back, dim3(nblk(n2, 256)), dim3(256), 0, st, Ot1, Ot2, OtT, O1, O2, no, nv,
                     accumulate ? 1 : 0);
}

__global__ void k_combine(const double* __restrict__ Ot1, const double* __restrict__ Ot2,
                          const double* __restrict__ OtT, double* __restrict__ O1,
                          double* __restrict__ O2, int no, int nv) {
  const int64_t nvl = nv, n2 = (int64_t)no * no * nvl * nvl;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n2) {
    const int b = (int)(e % nvl), a = (int)((e / nvl) % nvl);
    O2[e] = ot2(Ot2, OtT, (e / (nvl * nvl)) * nvl, nvl, a, b);
  }
  if (e < (int64_t)no * nv) O1[e] = Ot1[e];
}

void launch_combine(const double* Ot1, const double* Ot2, const double* OtT, double* O1,
                    double* O2, int no, int nv, hipStream_t st) {
  const int64_t n2 = (int64_t)no * no * nv * nv;
  hipLaunchKernelGGL(k_combine, dim3(nblk(n2, 256)), dim3(256), 0, st, Ot1, Ot2, OtT, O1, O2, no,
                     nv);
}

// ---------------------------------------------------------------------------
// Input checks (CC3_CHECK): pair symmetry of t2, symmetry of L in (p, q), and
// positive denominators (3 min e_vir - 3 max e_occ > 0).  Sets bits of *flag.
// ---------------------------------------------------------------------------
__device__ inline bool differs(double x, double y) {
  const double s = fmax(fabs(x), fabs(y));
  return fabs(x - y) > 1e-12 * s;
}

__global__ void k_check(const double* __restrict__ eps, const double* __restrict__ L,
                        const double* __restrict__ t2, int no, int nv, int nJ, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nvl = nv, n2 = (int64_t)no * no * nvl * nvl;
  int bits = 0;
  for (int64_t e = e0; e < n2; e += stride) {
    const int b = (int)(e % nvl), a = (int)((e / nvl) % nvl);
    const int j = (int)((e / (nvl * nvl)) % no), i = (int)(e / (nvl * nvl * no));
    if (differs(t2[e], t2[(((int64_t)j * no + i) * nvl + b) * nvl + a])) bits |= 1;
  }
  if (L) {
    const int64_t nmo = no + nv, nl = (int64_t)nJ * nmo * nmo;
    for (int64_t e = e0; e < nl; e += stride) {
      const int64_t q = e % nmo, pp = (e / nmo) % nmo, J = e / (nmo * nmo);
      if (differs(L[e], L[(J * nmo + q) * nmo + pp])) bits |= 2;
    }
  }
  if (e0 == 0) {
    double emax = eps[0], vmin = eps[no];
    for (int i = 1; i < no; ++i) emax = fmax(emax, eps[i]);
    for (int a = 1; a < nv; ++a) vmin = fmin(vmin, eps[no + a]);
    if (!(3.0 * vmin - 3.0 * emax > 0.0)) bits |= 4;
  }
  if (bits) atomicOr(flag, bits);
}

__global__ void k_zero_int(int* p) { *p = 0; }

void launch_check(const double* eps, const double* L, const double* t2, int no, int nv, int nJ,
                  int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, flag);
  hipLaunchKernelGGL(k_check, dim3(1024), dim3(256), 0, st, eps, L, t2, no, nv, nJ, flag);
}

}  // namespace cc3
