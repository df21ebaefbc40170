// Low-precision W build (the t3-building contractions of Algorithm 1's first
// statement) on gfx950 MFMA, with FP32 accumulation:
//   CC3_FP32   : v_mfma_f32_16x16x4f32 on FP32 copies of the operands;
//   CC3_BF16X3 : v_mfma_f32_16x16x32_bf16 on a 2-piece split x = hi + lo,
//                products hi*hi + hi*lo + lo*hi;
//   CC3_BF16X6 : 3-piece split x = hi + mid + lo, products hi*hi + hi*mid +
//                mid*hi + hi*lo + mid*mid + lo*hi.
// Each W term is accumulated in FP32 over its K range; the two terms of a plane
// are converted and summed in FP64 and the plane is stored in FP64, so the
// permutation sum, the denominator division, the contravariant combination
// and the Omega accumulation downstream stay FP64.
//
// The operands are re-laid out once per call so that the contracted index is
// contiguous and zero-padded to a multiple of 32 (tiles load as 16-byte
// chunks into row-major LDS rows, and the K loop needs no bounds checks):
//   t2L [piece][p][q][x][dk]  = t2[p][q][x][d]
//   t2NL[piece][p][y][x][lk]  = -t2[p][l][x][y]
//   GwTL[piece][r][y][z][dk]  = Gw[r][y][z][d]   (= g_{ydzr})
//   GoTL[piece][q][r][z][lk]  = Go[q][r][z][l]   (= g_{lqzr})
#include <hip/hip_bf16.h>

#include "cc3.h"
#include "cc3_device.hpp"
#include "cc3_internal.hpp"

namespace cc3 {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));  // a 16-byte chunk (kept in registers)

__host__ __device__ inline int kpad(int k) { return (k + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// Operand conversion: FP64 value -> pieces
// ---------------------------------------------------------------------------
// Generic re-layout: out[piece][outer][x][kk] (kk < K padded) from an FP64
// source element (outer, x, k) at src[outer * so + x * sx + k * sk] * sign.
// `piece_stride` is the element distance between pieces of the whole array.
template <int MODE>  // 0: FP32, 2: BF16 2-piece, 3: BF16 3-piece
__global__ void k_lp_copy(const double* __restrict__ src, int64_t so, int64_t sx, int64_t sk,
                          double sign, int nouter, int nx, int K, void* __restrict__ dst,
                          int64_t piece_stride) {
  const int Kp = kpad(K);
  const int64_t n = (int64_t)nouter * nx * Kp;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int kk = (int)(e % Kp);
  const int x = (int)((e / Kp) % nx);
  const int64_t o = e / ((int64_t)Kp * nx);
  const double v = (kk < K) ? sign * src[o * so + (int64_t)x * sx + (int64_t)kk * sk] : 0.0;
  if constexpr (MODE == 0) {
    ((float*)dst)[e] = (float)v;
  } else {
    constexpr int P = MODE;
    uint16_t pc[P];
    split_bf16<P>(v, pc);
#pragma unroll
    for (int i = 0; i < P; ++i) ((uint16_t*)dst)[i * piece_stride + e] = pc[i];
  }
}

static int mode_of(int prec) { return prec == CC3_FP32 ? 0 : prec == CC3_BF16X3 ? 2 : 3; }

size_t lp_operand_bytes(int prec, int no, int nv) {
  if (prec == CC3_FP64) return 0;
  const size_t o = no, v = nv, dk = kpad(nv), lk = kpad(no);
  const size_t elems = o * o * v * dk + o * v * v * lk + o * v * v * dk + o * o * v * lk;
  const size_t esz = prec == CC3_FP32 ? 4 : 2;
  const size_t pieces = prec == CC3_FP32 ? 1 : prec == CC3_BF16X3 ? 2 : 3;
  return elems * esz * pieces + 4 * 256;
}

void lp_operand_ptrs(int prec, int no, int nv, void* base, LpOperands& lp) {
  const size_t o = no, v = nv, dk = kpad(nv), lk = kpad(no);
  const size_t esz = prec == CC3_FP32 ? 4 : 2;
  const size_t pieces = prec == CC3_FP32 ? 1 : prec == CC3_BF16X3 ? 2 : 3;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* b = (char*)base;
  lp.t2 = b;
  b += al(o * o * v * dk * esz * pieces);
  lp.t2N = b;
  b += al(o * v * v * lk * esz * pieces);
  lp.GwT = b;
  b += al(o * v * v * dk * esz * pieces);
  lp.GoT = b;
  lp.prec = prec;
}

template <int MODE>
static void lp_copy(const double* src, int64_t so, int64_t sx, int64_t sk, double sign, int nouter,
                    int nx, int K, void* dst, int64_t piece_stride, hipStream_t st) {
  const int64_t n = (int64_t)nouter * nx * kpad(K);
  hipLaunchKernelGGL(k_lp_copy<MODE>, dim3(nblk(n, 256)), dim3(256), 0, st, src, so, sx, sk, sign,
                     nouter, nx, K, dst, piece_stride);
}

void launch_lp_convert(const double* t2, const Blocks& b, int no, int nv, const LpOperands& lp,
                       hipStream_t st) {
  const int64_t v = nv, o = no, dk = kpad(nv), lk = kpad(no);
  auto run = [&](auto mode_tag) {
    constexpr int M = decltype(mode_tag)::value;
    constexpr int64_t esz = (M == 0 ? 4 : 2);
    // t2L[p][q][x][d] = t2[p][q][x][d]
    lp_copy<M>(t2, v * v, v, 1, 1.0, no * no, nv, nv, lp.t2, o * o * v * dk, st);
    // t2NL[p][y][x][l] = -t2[p][l][x][y]: for each p, outer = y, x = x, k = l
    for (int p = 0; p < no; ++p)
      lp_copy<M>(t2 + (int64_t)p * o * v * v, 1, v, v * v, -1.0, nv, nv, no,
                 (char*)lp.t2N + (size_t)p * v * v * lk * esz, o * v * v * lk, st);
    // GwTL[r][y][z][d] = Gw[r][y][z][d]: outer = (r, y), x = z, k = d
    lp_copy<M>(b.Gw, v * v, v, 1, 1.0, no * nv, nv, nv, lp.GwT, o * v * v * dk, st);
    // GoTL[q][r][z][l] = Go[q][r][z][l]: outer = (q, r), x = z, k = l
    lp_copy<M>(b.Go, o * v, o, 1, 1.0, no * no, nv, no, lp.GoT, o * o * v * lk, st);
  };
  const int m = mode_of(lp.prec);
  if (m == 0) run(std::integral_constant<int, 0>());
  else if (m == 2) run(std::integral_constant<int, 2>());
  else run(std::integral_constant<int, 3>());
}

// ---------------------------------------------------------------------------
// W build in low precision
// ---------------------------------------------------------------------------
// 8 wavefronts as 4 (rows) x 2 (columns), each 32 x 64 outputs (2 x 4 blocks).
constexpr int LWM = 4, LWN = 2, LFM = 2, LFN = 4;
constexpr int LNT = 64 * LWM * LWN;
constexpr int LBM = 16 * LWM * LFM, LBN = 16 * LWN * LFN;  // 128 x 128

// Engine traits.  FLUSH: each LDS stage (32 k) is accumulated in FP32 from zero
// and then added into an FP64 accumulator, so the FP32 rounding of the MFMA
// outputs applies to 32-term partial sums rather than to the running sum over
// the whole K range.  Used where the split is fine enough for that rounding to
// dominate the error (FP32 and the 3-piece BF16 split); the 2-piece split is
// limited by its operands and keeps one FP32 accumulator per term.
// MINW: waves per SIMD the W kernel is built for (4: two workgroups per CU).
// NS: LDS stage buffers of the ring (NS - 1 stages of loads in flight).
struct EngF32 {
  static constexpr int BK = 32, P = 1, NPROD = 1, ESZ = 4;
  static constexpr bool FLUSH = true;
  static constexpr int MINW = 4, NS = 2;
};
template <int P_>
struct EngBF16 {
  static constexpr int BK = 32, P = P_, NPROD = (P_ == 2 ? 3 : 6), ESZ = 2;
  static constexpr bool FLUSH = (P_ == 3);
  static constexpr int MINW = (P_ == 2 ? 4 : 2), NS = (P_ == 2 ? 2 : 3);
};

// the piece pairs of the split products
__device__ inline void prod_pair(int P, int t, int& pa, int& pb) {
  if (P == 2) {
    const int a[3] = {0, 0, 1}, b[3] = {0, 1, 0};
    pa = a[t]; pb = b[t];
  } else {
    const int a[6] = {0, 0, 1, 0, 1, 2}, b[6] = {0, 1, 0, 2, 1, 0};
    pa = a[t]; pb = b[t];
  }
}

// ---------------------------------------------------------------------------
// The tile engine.  Operands are row-major (row, k) with k contiguous and
// zero-padded to a multiple of 32, in P pieces.  A stage holds 32 k of the
// 128 A rows and 128 B rows of every piece.  It goes from global memory to LDS
// directly: a buffer load with the LDS flag writes 16 bytes per lane at
// consecutive LDS addresses (1 KB per instruction), so the tile needs no
// staging registers and no LDS stores.  Each LDS row holds the RB bytes of one
// row and one stage as 16-byte chunks, XOR-swizzled by the row (lp_chunk) so
// that the 16 rows of one fragment read fall in different banks; the lane that
// fills LDS slot s loads the global chunk that the swizzle puts there.  Two
// stage buffers, one barrier per stage: the loads of stage s + 1 are issued
// before the MFMAs of stage s and waited for after them.
// ---------------------------------------------------------------------------
template <class E>
struct LpTile {
  static constexpr int P = E::P, ESZ = E::ESZ;
  static constexpr int RB = E::BK * ESZ;         // bytes of one row in one stage
  static constexpr int CPR = RB / 16;            // 16-byte chunks per row (8 or 4)
  static constexpr int TILEB = LBM * RB;         // one operand piece of one stage
  static constexpr int NI = TILEB / (LNT * 16);  // loads per lane per operand piece
  static constexpr int STAGEB = 2 * P * TILEB;
  static constexpr int NS = E::NS;               // stage buffers
  static constexpr int LPS = 2 * P * NI;         // direct loads per lane per stage
  static_assert(LBM == LBN && NI * LNT * 16 == TILEB, "tile shape");
  static_assert(NS >= 2 && (NS - 2) * LPS <= 63, "vmcnt range");
};

// LDS chunk of logical chunk c of row `row` (an involution in c).  Both forms
// measured free of bank conflicts (SQ_LDS_BANK_CONFLICT = 0) for the fragment
// reads, 16 rows by one chunk column per lane group; XOR with (row >> 2) & 3
// for 64-byte rows, or no swizzle, gives two-way conflicts.
template <class E>
__device__ inline int lp_chunk(int row, int c) {
  if constexpr (LpTile<E>::CPR == 8) return c ^ ((row >> 1) & 7);
  else return c ^ ((row >> 1) & 3);
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// One K segment of a product: piece-0 operand origins (row 0, k = 0), piece
// strides and row strides in bytes, and its number of stages.
struct LpSeg {
  const char *a, *b;
  int64_t aps, bps;
  unsigned ars, brs;
  int nst;
};

// The rows this lane loads: for load i of an operand piece, LDS slot
// s = (8 i + wave) 64 + lane holds row s / CPR and the swizzled chunk of s % CPR.
template <class E>
struct LpLanes {
  int row[LpTile<E>::NI];
  unsigned cb[LpTile<E>::NI];  // byte offset of the chunk within the row's stage
  __device__ LpLanes(int wave, int lane) {
    typedef LpTile<E> L;
#pragma unroll
    for (int i = 0; i < L::NI; ++i) {
      const int s = (8 * i + wave) * 64 + lane;
      row[i] = s / L::CPR;
      cb[i] = (unsigned)lp_chunk<E>(row[i], s % L::CPR) * 16u;
    }
  }
};

// Issue the direct loads of stage `st` of segment `sg` into the stage buffer
// `buf`; ar / br: this lane's A and B row indices (already mapped to operand rows)
template <class E>
__device__ __forceinline__ void lp_load_stage(const LpSeg& sg, int st, char* buf,
                                              const unsigned* cb, const int* ar, const int* br,
                                              int wave) {
  typedef LpTile<E> L;
  const int64_t ko = (int64_t)st * L::RB;
#pragma unroll
  for (int pc = 0; pc < L::P; ++pc) {
    const BufRsrc ra = buf_rsrc(sg.a + pc * sg.aps + ko), rb = buf_rsrc(sg.b + pc * sg.bps + ko);
#pragma unroll
    for (int i = 0; i < L::NI; ++i) {
      char* la = buf + pc * L::TILEB + (8 * i + wave) * 1024;
      char* lb = buf + (L::P + pc) * L::TILEB + (8 * i + wave) * 1024;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_t)la, 16,
                                               (unsigned)ar[i] * sg.ars + cb[i], 0, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr_t)lb, 16,
                                               (unsigned)br[i] * sg.brs + cb[i], 0, 0, 0);
    }
  }
}

// The oldest stage in flight has reached LDS for every lane: this lane waits until at
// most `later` stages of its loads are outstanding (they return in order), then the
// workgroup barrier.  The barrier also ends every wave's reads of the previous stage,
// whose buffer the next loads overwrite.
template <int N>
__device__ __forceinline__ void lp_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
template <class E>
__device__ __forceinline__ void lp_stage_ready(int later) {
  typedef LpTile<E> L;
  if constexpr (L::NS >= 3) {
    if (later >= 1) {
      if constexpr (L::NS >= 4) {
        if (later >= 2) {
          lp_vmcnt<2 * L::LPS>();
          __syncthreads();
          return;
        }
      }
      lp_vmcnt<L::LPS>();
      __syncthreads();
      return;
    }
  }
  lp_vmcnt<0>();
  __syncthreads();
}

// acc += A B over one LDS stage.  BF16: one k = 32 MFMA per product; lane
// supplies A[m = l%16][k = 8 (l/16) .. + 7] (chunk l/16 of its row).  FP32: the
// lane reads chunk 4 h + l/16 (four consecutive k) of its row and supplies its
// element j to the k-step (h, j) of the 16x16x4 MFMA; A and B use the same k
// assignment, so the eight k-steps cover the stage's 32 k once each.
template <class E>
__device__ __forceinline__ void lp_mfma_stage(const char* buf, f4v (&acc)[LFM][LFN], int lane,
                                              int wm, int wn) {
  typedef LpTile<E> L;
  const int g = lane >> 4, r16 = lane & 15;
  // Fragment rows are 16 R + r16, and lp_chunk's XOR depends on bits 1-3 of the row
  // only, that is on r16: the lane's byte offset within a fragment's rows is one value
  // per chunk column, and the fragment's own offset (16 R RB) is a constant.
  auto lane_off = [&](int c) __attribute__((always_inline)) {
    return r16 * L::RB + lp_chunk<E>(r16, c) * 16;
  };
  const char* ab = buf + wm * LFM * 16 * L::RB;             // this wave's A rows
  const char* bb = buf + L::P * L::TILEB + wn * LFN * 16 * L::RB;  // and B rows
  if constexpr (E::P == 1) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lo = lane_off(4 * h + g);
      f4v a[LFM];
#pragma unroll
      for (int fm = 0; fm < LFM; ++fm) a[fm] = *(const f4v*)(ab + fm * 16 * L::RB + lo);
      // one B fragment at a time (registers: the FP64 accumulator of FLUSH is large)
#pragma unroll
      for (int fn = 0; fn < LFN; ++fn) {
        const f4v b = *(const f4v*)(bb + fn * 16 * L::RB + lo);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int fm = 0; fm < LFM; ++fm)
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[fm][j], b[j], acc[fm][fn], 0, 0, 0);
      }
    }
  } else {
    const int lo = lane_off(g);
    bf8v a[L::P][LFM], b[L::P][LFN];
#pragma unroll
    for (int pc = 0; pc < L::P; ++pc) {
#pragma unroll
      for (int fm = 0; fm < LFM; ++fm)
        a[pc][fm] = *(const bf8v*)(ab + pc * L::TILEB + fm * 16 * L::RB + lo);
#pragma unroll
      for (int fn = 0; fn < LFN; ++fn)
        b[pc][fn] = *(const bf8v*)(bb + pc * L::TILEB + fn * 16 * L::RB + lo);
    }
#pragma unroll
    for (int t = 0; t < E::NPROD; ++t) {
      int pa, pb;
      prod_pair(L::P, t, pa, pb);
#pragma unroll
      for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
        for (int fn = 0; fn < LFN; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[pa][fm], b[pb][fn], acc[fm][fn], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void lp_zero(f4v (&acc)[LFM][LFN]) {
#pragma unroll
  for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
    for (int fn = 0; fn < LFN; ++fn) acc[fm][fn] = f4v{0.f, 0.f, 0.f, 0.f};
}
__device__ __forceinline__ void lp_flush(f4v (&acc)[LFM][LFN], d4v (&accd)[LFM][LFN]) {
#pragma unroll
  for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
    for (int fn = 0; fn < LFN; ++fn) {
#pragma unroll
      for (int r = 0; r < 4; ++r) accd[fm][fn][r] += (double)acc[fm][fn][r];
      acc[fm][fn] = f4v{0.f, 0.f, 0.f, 0.f};
    }
}

// ---------------------------------------------------------------------------
// W build in low precision
// ---------------------------------------------------------------------------
// Issue the loads of stage t of the plane (its four K segments in turn) into buf.
// The segments are passed by value and each call site names one of them, so that they
// stay in scalar registers.
template <class E>
__device__ __forceinline__ void wlp_load(int t, char* buf, const LpSeg s0, const LpSeg s1,
                                         const LpSeg s2, const LpSeg s3, const unsigned* cb,
                                         const int* ar, const int* br, int wave) {
  if (t < s0.nst) { lp_load_stage<E>(s0, t, buf, cb, ar, br, wave); return; }
  t -= s0.nst;
  if (t < s1.nst) { lp_load_stage<E>(s1, t, buf, cb, ar, br, wave); return; }
  t -= s1.nst;
  if (t < s2.nst) { lp_load_stage<E>(s2, t, buf, cb, ar, br, wave); return; }
  t -= s2.nst;
  lp_load_stage<E>(s3, t, buf, cb, ar, br, wave);
}

// Stages [sb, se) of the plane's nsteps into acc (with FLUSH into accd), the loads
// running NS - 1 stages ahead in the ring of NS stage buffers.
template <class E>
__device__ __forceinline__ void wlp_run(int sb, int se, int nsteps, char* lds, const LpSeg s0,
                                        const LpSeg s1, const LpSeg s2, const LpSeg s3,
                                        const unsigned* cb, const int* ar, const int* br,
                                        int wave, int lane, int wm, int wn,
                                        f4v (&acc)[LFM][LFN], d4v (&accd)[LFM][LFN]) {
  typedef LpTile<E> L;
  for (int s = sb; s < se; ++s) {
    lp_stage_ready<E>(min(L::NS - 2, nsteps - 1 - s));
    const int ahead = s + L::NS - 1;
    if (ahead < nsteps)
      wlp_load<E>(ahead, lds + (ahead % L::NS) * L::STAGEB, s0, s1, s2, s3, cb, ar, br, wave);
    lp_mfma_stage<E>(lds + (s % L::NS) * L::STAGEB, acc, lane, wm, wn);
    if constexpr (E::FLUSH) lp_flush(acc, accd);
  }
}

template <class E>
__device__ __forceinline__ void wbuild_lp_body(
    const char* __restrict__ t2L, const char* __restrict__ t2NL, const char* __restrict__ GwTL,
    const char* __restrict__ GoTL, const int* __restrict__ tri, double* __restrict__ cubes, int no,
    int nv, int tiles_m, int tiles_n, int all_terms, int bx, int by, int bz) {
  typedef LpTile<E> L;
  constexpr int ESZ = E::ESZ;
  __shared__ __attribute__((aligned(16))) char lds[L::NS * L::STAGEB];
  const int tpp = tiles_m * tiles_n;
  const int y = bx / tpp;
  const int tile = bx % tpp;
  const int m0 = (tile / tiles_n) * LBM, n0 = (tile % tiles_n) * LBN;
  const int plane = by;
  const int z = bz;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  int kind = (i == j) ? 1 : (j == k) ? 2 : 0;
  if (all_terms) kind = 0;
  if ((kind == 1 && plane == 1) || (kind == 2 && plane == 2)) return;
  const bool two = (kind == 0) || plane == 0;
  int p1, q1, r1, p2, q2, r2;
  if (plane == 0) { p1 = i; q1 = j; r1 = k; p2 = k; q2 = j; r2 = i; }
  else if (plane == 1) { p1 = j; q1 = i; r1 = k; p2 = k; q2 = i; r2 = j; }
  else { p1 = i; q1 = k; r1 = j; p2 = j; q2 = k; r2 = i; }

  const int64_t dk = kpad(nv), lk = kpad(no), v = nv, o = no;
  // piece strides (bytes) of the four arrays
  const int64_t ps_t2 = o * o * v * dk * ESZ, ps_t2N = o * v * v * lk * ESZ,
                ps_Gw = o * v * v * dk * ESZ, ps_Go = o * o * v * lk * ESZ;
  const unsigned rv = (unsigned)(dk * ESZ), ro = (unsigned)(lk * ESZ);
  // segments: term 1 vv, term 1 oo, term 2 vv, term 2 oo (rows m for A, n for B)
  // segments: term 1 vv, term 1 oo, term 2 vv, term 2 oo (rows m for A, n for B)
  const LpSeg sg0 = {t2L + ((p1 * o + q1) * v) * dk * ESZ, GwTL + ((r1 * v + y) * v) * dk * ESZ,
                     ps_t2, ps_Gw, rv, rv, (int)(dk / 32)};
  const LpSeg sg1 = {t2NL + ((p1 * v + y) * v) * lk * ESZ, GoTL + ((q1 * o + r1) * v) * lk * ESZ,
                     ps_t2N, ps_Go, ro, ro, (int)(lk / 32)};
  const LpSeg sg2 = {GwTL + ((r2 * v + y) * v) * dk * ESZ, t2L + ((p2 * o + q2) * v) * dk * ESZ,
                     ps_Gw, ps_t2, rv, rv, (int)(dk / 32)};
  const LpSeg sg3 = {GoTL + ((q2 * o + r2) * v) * lk * ESZ, t2NL + ((p2 * v + y) * v) * lk * ESZ,
                     ps_Go, ps_t2N, ro, ro, (int)(lk / 32)};

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % LWM, wn = wave / LWM;
  const LpLanes<E> ln(wave, lane);
  // rows past nv repeat row nv - 1 (their outputs are never stored)
  int ar[L::NI], br[L::NI];
#pragma unroll
  for (int e = 0; e < L::NI; ++e) {
    ar[e] = min(m0 + ln.row[e], nv - 1);
    br[e] = min(n0 + ln.row[e], nv - 1);
  }

  // term 1 (and term 2 when the plane has two), each accumulated in FP32 (with
  // FLUSH stage by stage into FP64); the plane value is their FP64 sum
  f4v acc1[LFM][LFN], acc2[LFM][LFN];
  d4v accd[LFM][LFN];
  lp_zero(acc1);
  lp_zero(acc2);
#pragma unroll
  for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
    for (int fn = 0; fn < LFN; ++fn) accd[fm][fn] = d4v{0.0, 0.0, 0.0, 0.0};
  const int nt1 = sg0.nst + sg1.nst;  // stages of one term
  const int nsteps = two ? 2 * nt1 : nt1;
#pragma unroll
  for (int t = 0; t < L::NS - 1; ++t)
    if (t < nsteps) wlp_load<E>(t, lds + t * L::STAGEB, sg0, sg1, sg2, sg3, ln.cb, ar, br, wave);
  wlp_run<E>(0, nt1, nsteps, lds, sg0, sg1, sg2, sg3, ln.cb, ar, br, wave, lane, wm, wn, acc1, accd);
  if (two) {
    f4v (&acc)[LFM][LFN] = E::FLUSH ? acc1 : acc2;
    wlp_run<E>(nt1, nsteps, nsteps, lds, sg0, sg1, sg2, sg3, ln.cb, ar, br, wave, lane, wm, wn,
               acc, accd);
  }

  // the FP32/BF16 MFMA leaves D[row = 4 (lane/16) + r][col = lane%16] in register r
  // the padded rows of the triple loop's cubes
  const int64_t rp = cube_pitch(nv);
  double* dst = cubes + ((int64_t)z * 5 + plane) * cube_slot(nv) + (int64_t)y * nv * rp;
#pragma unroll
  for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
    for (int fn = 0; fn < LFN; ++fn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + (wm * LFM + fm) * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + (wn * LFN + fn) * 16 + (lane & 15);
        if (m < nv && n < nv)
          dst[(int64_t)m * rp + n] = accd[fm][fn][r] + ((double)acc1[fm][fn][r] + (double)acc2[fm][fn][r]);
      }
}

template <class E>
__global__ __launch_bounds__(LNT, E::MINW) void k_wbuild_lp(
    const char* __restrict__ t2L, const char* __restrict__ t2NL, const char* __restrict__ GwTL,
    const char* __restrict__ GoTL, const int* __restrict__ tri, double* __restrict__ cubes, int no,
    int nv, int tiles_m, int tiles_n, int all_terms) {
  wbuild_lp_body<E>(t2L, t2NL, GwTL, GoTL, tri, cubes, no, nv, tiles_m, tiles_n, all_terms,
                    blockIdx.x, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------------------
// Mixed-all Omega contraction (the vv term and Omega1) on split-BF16 MFMA
// ---------------------------------------------------------------------------
// The long-K GEMM of k_omega per (triple, permutation, 128 x 128 tile, K chunk):
//   Pvv[z][pi][chunk][a][n] = sum_{kk in chunk} Y_v(pi)[a][kk] G[r][n'][kk],
// with every operand row k-contiguous, K = (x, y) in the blocked order lp_kb (8 x 8
// blocks of 64 contiguous values, Kp = lp_kb_len(nv), zero where x or y >= nv):
//   YL[z][v][piece][a][kk]: the four k-major views of tau~ that the six
//     permutations need, kk = lp_kb(x, y), written by k_mix:
//     v = 0: tau~[a][x][y] (pi 0);  1: tau~[x][a][y] (pi 1, 4);
//     v = 2: tau~[x][y][a] (pi 2, 5);  3: tau~[a][y][x] (pi 3);
//   GL[piece][r][n'][kk]: Gbc (or Gcb for pi 2, 4) rows, n' = n for n < nv and
//     nv + q (the Omega1 row) for n >= nv.
// Each chunk sums in FP32 on the MFMA (with FLUSH, stage by stage into FP64);
// k_reduce sums the chunks in FP64.  The tile engine is that of k_wbuild_lp.
template <class E>
__global__ __launch_bounds__(LNT) void k_omega_lp(const char* __restrict__ YL,
                                                  const char* __restrict__ GbcL,
                                                  const char* __restrict__ GcbL,
                                                  const int* __restrict__ tri,
                                                  double* __restrict__ Pvv, int no, int nv,
                                                  int nchunks, int tiles_n) {
  typedef LpTile<E> L;
  constexpr int ESZ = E::ESZ;
  __shared__ __attribute__((aligned(16))) char lds[L::NS * L::STAGEB];
  const int pi = blockIdx.y, z = blockIdx.z;
  const int i = tri[3 * z], j = tri[3 * z + 1], k = tri[3 * z + 2];
  if (!perm_active(tri_kind(i, j, k), pi)) return;
  int p, q, r;
  perm_pqr(pi, i, j, k, p, q, r);
  const int ch = blockIdx.x % nchunks, tile = blockIdx.x / nchunks;
  const int m0 = (tile / tiles_n) * LBM, n0 = (tile % tiles_n) * LBN;
  const int64_t Kp = lp_kb_len(nv);  // the blocked K of the views and of GL
  const int S = (int)(Kp / E::BK);
  const int64_t Kr = lp_kb_pitch(nv);  // their row pitch
  const int s0 = (int)((int64_t)ch * S / nchunks), s1 = (int)((int64_t)(ch + 1) * S / nchunks);
  if (s0 >= s1) return;
  const int view = pi == 0 ? 0 : pi == 3 ? 3 : (pi == 1 || pi == 4) ? 1 : 2;
  const bool cb = (pi == 2 || pi == 4);
  const int64_t rs = Kr * ESZ;                                   // row stride, bytes
  const int64_t y_ps = (int64_t)nv * rs;                         // piece stride of a view
  const int64_t g_ps = (int64_t)no * (nv + no) * rs;             // piece stride of GL
  const LpSeg sg = {YL + ((int64_t)z * 4 + view) * E::P * y_ps,
                    (cb ? GcbL : GbcL) + (int64_t)r * (nv + no) * rs, y_ps, g_ps,
                    (unsigned)rs, (unsigned)rs, S};

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % LWM, wn = wave / LWM;
  const LpLanes<E> ln(wave, lane);
  // rows past nv repeat row nv - 1 (outputs never stored); B rows n >= nv read the
  // Omega1 row nv + q
  int ar[L::NI], br[L::NI];
#pragma unroll
  for (int e = 0; e < L::NI; ++e) {
    ar[e] = min(m0 + ln.row[e], nv - 1);
    const int n = n0 + ln.row[e];
    br[e] = n < nv ? n : nv + q;
  }
  f4v acc[LFM][LFN];
  d4v accd[LFM][LFN];  // FLUSH: each stage's FP32 sum added in FP64
  lp_zero(acc);
#pragma unroll
  for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
    for (int fn = 0; fn < LFN; ++fn) accd[fm][fn] = d4v{0.0, 0.0, 0.0, 0.0};
  // the loads run NS - 1 stages ahead in the ring of NS stage buffers
#pragma unroll
  for (int t = 0; t < L::NS - 1; ++t)
    if (s0 + t < s1) lp_load_stage<E>(sg, s0 + t, lds + t * L::STAGEB, ln.cb, ar, br, wave);
  for (int s = s0; s < s1; ++s) {
    lp_stage_ready<E>(min(L::NS - 2, s1 - 1 - s));
    const int ahead = s - s0 + L::NS - 1;
    if (s0 + ahead < s1)
      lp_load_stage<E>(sg, s0 + ahead, lds + (ahead % L::NS) * L::STAGEB, ln.cb, ar, br, wave);
    lp_mfma_stage<E>(lds + ((s - s0) % L::NS) * L::STAGEB, acc, lane, wm, wn);
    if constexpr (E::FLUSH) lp_flush(acc, accd);
  }
  // the BF16 MFMA leaves D[row = 4 (lane/16) + r][col = lane%16] in register r
  const int NV1 = nv + 1;
  double* pvv = Pvv + (((int64_t)z * 6 + pi) * nchunks + ch) * (int64_t)nv * NV1;
#pragma unroll
  for (int fm = 0; fm < LFM; ++fm)
#pragma unroll
    for (int fn = 0; fn < LFN; ++fn)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = m0 + (wm * LFM + fm) * 16 + 4 * (lane >> 4) + rr;
        const int n = n0 + (wn * LFN + fn) * 16 + (lane & 15);
        if (a < nv && n <= nv) pvv[(int64_t)a * NV1 + n] = accd[fm][fn][rr] + (double)acc[fm][fn][rr];
      }
}

// Zero n 16-bit values (the YL views, whose blocked K positions with an index past nv
// k_mix never writes), 8 per thread and pass.
__global__ void k_zero_pad(uint16_t* __restrict__ p, int64_t n) {
  const int64_t n8 = n / 8;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n8;
       e += (int64_t)gridDim.x * blockDim.x)
    ((uint4*)p)[e] = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t e = n8 * 8 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0;
}

void launch_lp_zero_pad(void* YL, int64_t rows, int nv, hipStream_t st) {
  if (nv % 8 == 0 || rows == 0) return;  // no position of the blocked K lies past nv
  const int64_t n = rows * lp_kb_pitch(nv);
  unsigned g = nblk(n / 8 + 1, 256);
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_zero_pad, dim3(g), dim3(256), 0, st, (uint16_t*)YL, n);
}

size_t lp_contract_g_bytes(int prec, int no, int nv) {
  const int P = prec == CC3_BF16X3 ? 2 : 3;
  return (size_t)P * no * (nv + no) * (size_t)lp_kb_pitch(nv) * 2;  // one of Gbc, Gcb
}
size_t lp_contract_cube_bytes(int prec, int nv) {
  const int P = prec == CC3_BF16X3 ? 2 : 3;
  return (size_t)4 * P * nv * (size_t)lp_kb_pitch(nv) * 2;  // per triple
}

// Split-BF16 pieces of the rows of Gbc or Gcb with K = (x, y) (x nv + y in the source)
// in the blocked order lp_kb: dst[piece][row][kb] at row pitch lp_kb_pitch, zero where x
// or y is past nv (the pitch's tail is never read).
template <int P>
__global__ void k_lp_copy_blocked(const double* __restrict__ src, int64_t rows, int nv,
                                  uint16_t* __restrict__ dst, int64_t piece_stride) {
  const int64_t Kb = lp_kb_len(nv), Kr = lp_kb_pitch(nv), K = (int64_t)nv * nv;
  const int nb = (nv + 7) / 8;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * Kb) return;
  const int64_t row = e / Kb;
  const int kb = (int)(e % Kb);
  const int blk = kb >> 6, x = (blk / nb) * 8 + ((kb >> 3) & 7), y = (blk % nb) * 8 + (kb & 7);
  const double v = (x < nv && y < nv) ? src[row * K + (int64_t)x * nv + y] : 0.0;
  uint16_t pc[P];
  split_bf16<P>(v, pc);
#pragma unroll
  for (int i = 0; i < P; ++i) dst[i * piece_stride + row * Kr + kb] = pc[i];
}

void launch_lp_contract_convert(const Blocks& b, int prec, int no, int nv, void* GbcL, void* GcbL,
                                hipStream_t st) {
  const int64_t rows = (int64_t)no * (nv + no), n = rows * lp_kb_len(nv);
  const int64_t ps = rows * lp_kb_pitch(nv);  // piece stride (elements)
  const unsigned g = nblk(n, 256);
  if (prec == CC3_BF16X3) {
    hipLaunchKernelGGL(k_lp_copy_blocked<2>, dim3(g), dim3(256), 0, st, b.Gbc, rows, nv,
                       (uint16_t*)GbcL, ps);
    hipLaunchKernelGGL(k_lp_copy_blocked<2>, dim3(g), dim3(256), 0, st, b.Gcb, rows, nv,
                       (uint16_t*)GcbL, ps);
  } else {
    hipLaunchKernelGGL(k_lp_copy_blocked<3>, dim3(g), dim3(256), 0, st, b.Gbc, rows, nv,
                       (uint16_t*)GbcL, ps);
    hipLaunchKernelGGL(k_lp_copy_blocked<3>, dim3(g), dim3(256), 0, st, b.Gcb, rows, nv,
                       (uint16_t*)GcbL, ps);
  }
}

void launch_omega_lp(int prec, const void* YL, const void* GbcL, const void* GcbL, const int* tri,
                     int ntri, double* Pvv, int no, int nv, hipStream_t st) {
  const int tm = (nv + LBM - 1) / LBM, tn = (nv + 1 + LBN - 1) / LBN;
  const int nch = omega_kchunks(nv, ntri, true);
  const dim3 grid(nch * tm * tn, 6, ntri), block(LNT);
  const char *y = (const char*)YL, *gb = (const char*)GbcL, *gc = (const char*)GcbL;
  if (prec == CC3_BF16X3)
    hipLaunchKernelGGL(k_omega_lp<EngBF16<2>>, grid, block, 0, st, y, gb, gc, tri, Pvv, no, nv, nch, tn);
  else
    hipLaunchKernelGGL(k_omega_lp<EngBF16<3>>, grid, block, 0, st, y, gb, gc, tri, Pvv, no, nv, nch, tn);
}

// Packed persistent form of the low-precision W build (serving), as k_pack_wbuild.
template <class E>
__global__ __launch_bounds__(LNT) void k_pack_wbuild_lp(const PackJob* __restrict__ jobs,
                                                        int njobs, unsigned total) {
  for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
    int r = 0;
    while (r + 1 < njobs && item >= jobs[r + 1].first[PK_W]) ++r;
    const PackJob& J = jobs[r];
    const unsigned local = item - J.first[PK_W];
    const int tm = (J.nv + LBM - 1) / LBM, tn = (J.nv + LBN - 1) / LBN;
    const unsigned gx = (unsigned)J.nv * tm * tn;
    wbuild_lp_body<E>((const char*)J.lpt2, (const char*)J.lpt2N, (const char*)J.lpGwT,
                      (const char*)J.lpGoT, J.tri, J.cubes, J.no, J.nv, tm, tn, 0,
                      (int)(local % gx), (int)((local / gx) % 3), (int)(local / (gx * 3)));
    __syncthreads();
  }
}

void launch_wbuild_lp_packed(const PackJob* jobs, int njobs, unsigned total, int prec,
                             hipStream_t st) {
  const dim3 grid(total < 2048 ? total : 2048), block(LNT);
  if (prec == CC3_FP32)
    hipLaunchKernelGGL(k_pack_wbuild_lp<EngF32>, grid, block, 0, st, jobs, njobs, total);
  else if (prec == CC3_BF16X3)
    hipLaunchKernelGGL(k_pack_wbuild_lp<EngBF16<2>>, grid, block, 0, st, jobs, njobs, total);
  else
    hipLaunchKernelGGL(k_pack_wbuild_lp<EngBF16<3>>, grid, block, 0, st, jobs, njobs, total);
}

void launch_wbuild_lp(const LpOperands& lp, const int* tri, int ntri, double* cubes, int no, int nv,
                      bool all_terms, hipStream_t st) {
  const int tm = (nv + LBM - 1) / LBM, tn = (nv + LBN - 1) / LBN;
  const dim3 grid(nv * tm * tn, 3, ntri), block(LNT);
  const char *a = (const char*)lp.t2, *b = (const char*)lp.t2N, *c = (const char*)lp.GwT,
             *d = (const char*)lp.GoT;
  const int at = all_terms ? 1 : 0;
  if (lp.prec == CC3_FP32)
    hipLaunchKernelGGL(k_wbuild_lp<EngF32>, grid, block, 0, st, a, b, c, d, tri, cubes, no, nv, tm, tn, at);
  else if (lp.prec == CC3_BF16X3)
    hipLaunchKernelGGL(k_wbuild_lp<EngBF16<2>>, grid, block, 0, st, a, b, c, d, tri, cubes, no, nv, tm, tn, at);
  else
    hipLaunchKernelGGL(k_wbuild_lp<EngBF16<3>>, grid, block, 0, st, a, b, c, d, tri, cubes, no, nv, tm, tn, at);
}

}  // namespace cc3
