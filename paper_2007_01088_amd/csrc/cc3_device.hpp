// Device-side building blocks shared by the gfx950 kernels of libcc3: the
// FP64 MFMA tile engine (v_mfma_f64_16x16x4f64, 64-wide wavefronts, LDS-staged
// operands with register prefetch and double-buffered LDS).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc3 {

typedef double d4v __attribute__((ext_vector_type(4)));

// A strided 2D operand view: element (x, k) lives at p[x * sx + k * sk]; outside
// [0, xlim) x [0, klim) it reads as zero.  `xfast` selects the thread mapping
// of the global loads: true when x is the contiguous index, false when k is.
// Offsets relative to p must fit in 32 bits (p itself is 64-bit).
struct Opnd {
  const double* p;
  int sx, sk;
  int xlim, klim;
  bool xfast;
};

__device__ inline Opnd make_opnd(const double* p, int64_t sx, int64_t sk, int xlim, int klim,
                                 bool xfast) {
  Opnd o;
  o.p = p; o.sx = (int)sx; o.sk = (int)sk; o.xlim = xlim; o.klim = klim; o.xfast = xfast;
  return o;
}

// Raw buffer access: a resource for a uniform base pointer (range 2 GiB, no
// stride) and 64-bit loads at 32-bit per-lane byte offsets.
typedef __amdgpu_buffer_rsrc_t BufRsrc;
typedef unsigned u2v_ __attribute__((ext_vector_type(2)));
__device__ inline BufRsrc buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
__device__ inline double buf_load_f64(BufRsrc r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Split of an FP64 value into BF16 pieces (the low-precision forms):
// bf16_rn rounds to the nearest BF16, ties to even.
__device__ inline uint16_t bf16_rn(double x) {
  // round-to-nearest-even of the FP32 rounding of x (x is representable after
  // the first rounding to FP32 for the magnitudes of the pieces used here)
  const float f = (float)x;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_val(uint16_t h) { return (double)__uint_as_float(((uint32_t)h) << 16); }

// pieces of x: piece 0 = hi, 1 = next, 2 = last (BF16); FP32 uses one float
template <int P>
__device__ inline void split_bf16(double x, uint16_t (&pc)[P]) {
  double rest = x;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    pc[i] = bf16_rn(rest);
    rest -= bf16_val(pc[i]);
  }
}


// Tile geometry: WM x WN wavefronts, each owning FM x FN blocks of 16x16
// outputs; BK (a multiple of 4) k values per LDS stage.
template <int WM_, int WN_, int FM_, int FN_, int BK_ = 8>
struct TileCfg {
  static constexpr int WM = WM_, WN = WN_, FM = FM_, FN = FN_;
  static constexpr int NW = WM * WN;
  static constexpr int NT = 64 * NW;
  static constexpr int BM = 16 * WM * FM;
  static constexpr int BN = 16 * WN * FN;
  static constexpr int BK = BK_;
  static constexpr int LDA = BM;  // k-major LDS tiles, XOR-swizzled (see lds_idx)
  static constexpr int LDB = BN;
  static constexpr int EA = (BM * BK + NT - 1) / NT;
  static constexpr int EB = (BN * BK + NT - 1) / NT;
  static constexpr int STAGE = BK * (LDA + LDB);  // doubles per LDS stage
  static constexpr int LDS_DOUBLES = 2 * STAGE;
};

// LDS position of tile element (k, x) of a stage with BK rows: row k, with the
// low four bits of x XOR-ed by a k-dependent pattern that spreads the BK rows
// over the 16 slots of a 128-byte group (k for BK = 16, 2k for BK = 8, k mod 16
// for BK = 32).  A
// fragment read (16 consecutive x of one row) stays a permutation of one
// 128-byte group; a k-fast store (16 lanes covering BK rows and 16/BK adjacent
// x) lands on 16 different 8-byte bank pairs instead of one.
template <int BK>
__device__ inline int lds_swz(int k) {
  if constexpr (BK >= 16) return k & 15;  // BK = 32: rows k and k + 16 share a pattern
  else return (k & (BK - 1)) * (16 / BK);
}
template <int BK>
__device__ inline int lds_idx(int k, int x, int ld) { return k * ld + (x ^ lds_swz<BK>(k)); }

// Per-thread element mapping of an (X x BK) stage: element e of thread `tid`
// sits at (x_t + e*dx, k_t + e*dk).
template <int X, int BK, int NT>
struct StageMap {
  static_assert(NT % BK == 0, "BK must divide the thread count");
  static_assert(BK == 4 || BK == 8 || BK == 16 || BK == 32, "BK must be 4, 8, 16 or 32");
  static constexpr bool XF_OK = (NT % X == 0);  // x-fast mapping keeps x fixed per thread
  int x_t, k_t, dx, dk;
  __device__ StageMap(bool xfast, int tid) {
    if (xfast && XF_OK) { x_t = tid % X; k_t = tid / X; dx = 0; dk = NT / X; }
    else { k_t = tid % BK; x_t = tid / BK; dx = NT / BK; dk = 0; }
  }
};

// Global -> registers for one (X x BK) stage of an operand; x0/k0 the tile origin.
// Elements outside the operand load its first element instead, and bit e of zm
// tells which elements are inside: their zero is applied by store_stage, after
// the current stage's MFMAs, so that the loads stay in flight during them.
template <int X, int BK, int E, int NT>
__device__ inline void load_stage(const Opnd& o, int x0, int k0, double (&r)[E], unsigned& zm,
                                  int tid) {
  const StageMap<X, BK, NT> mp(o.xfast, tid);
  const double* base = o.p + ((int64_t)x0 * o.sx + (int64_t)k0 * o.sk);
  const int off0 = mp.x_t * o.sx + mp.k_t * o.sk;
  const int step = mp.dx * o.sx + mp.dk * o.sk;
  const bool interior = (x0 + X <= o.xlim) && (k0 + BK <= o.klim);
  zm = 0u;
  if (interior) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool in = (e * NT + tid) < X * BK;
      r[e] = *(in ? base + off0 + e * step : o.p);
      zm |= in ? (1u << e) : 0u;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int x = x0 + mp.x_t + e * mp.dx, k = k0 + mp.k_t + e * mp.dk;
      const bool in = (e * NT + tid) < X * BK && x < o.xlim && k < o.klim;
      r[e] = *(in ? base + off0 + e * step : o.p);
      zm |= in ? (1u << e) : 0u;
    }
  }
}

// Registers -> swizzled k-major LDS tile (same element mapping as load_stage);
// elements outside the operand (zm bit clear) are stored as zero.
template <int X, int BK, int E, int NT, int LD>
__device__ inline void store_stage(bool xfast, const double (&r)[E], unsigned zm, double* s,
                                   int tid) {
  const StageMap<X, BK, NT> mp(xfast, tid);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if ((e * NT + tid) < X * BK)
      s[lds_idx<BK>(mp.k_t + e * mp.dk, mp.x_t + e * mp.dx, LD)] = ((zm >> e) & 1u) ? r[e] : 0.0;
  }
}

// acc += A_tile * B_tile for one LDS stage.  A stage at sa (k-major, LDA),
// B stage at sb (k-major, LDB).  Lane l of a wave supplies A[m = l%16][k = l/16]
// and B[k = l/16][n = l%16] to each 16x16x4 FP64 MFMA.
template <class T>
__device__ inline void mfma_stage(const double* sa, const double* sb, d4v (&acc)[T::FM][T::FN],
                                  int lane, int wm, int wn) {
#pragma unroll
  for (int kk = 0; kk < T::BK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    const int sw = (lane & 15) ^ lds_swz<T::BK>(kr);
    double a[T::FM], b[T::FN];
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm) a[fm] = sa[kr * T::LDA + (wm * T::FM + fm) * 16 + sw];
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn) b[fn] = sb[kr * T::LDB + (wn * T::FN + fn) * 16 + sw];
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < T::FN; ++fn)
        acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
  }
}

// Output coordinate of accumulator element (fm, fn, r) for this lane:
// the FP64 16x16x4 MFMA leaves D[row = lane/16 + 4r][col = lane%16] in register r.
template <class T>
__device__ inline int acc_row(int wm, int fm, int lane, int r) {
  return (wm * T::FM + fm) * 16 + (lane >> 4) + 4 * r;
}
template <class T>
__device__ inline int acc_col(int wn, int fn, int lane) {
  return (wn * T::FN + fn) * 16 + (lane & 15);
}

template <class T>
__device__ inline void zero_acc(d4v (&acc)[T::FM][T::FN]) {
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn) acc[fm][fn] = d4v{0.0, 0.0, 0.0, 0.0};
}

// The K loop: `ops(step, A, B, k0)` fills the operand views of K step `step`
// (k0 = first k of the step within its operands).  Double-buffered LDS with
// one barrier per step; the next stage's global loads are in flight during the
// current stage's MFMAs.
template <class T, class Ops>
__device__ inline void k_loop(int nsteps, int m0, int n0, Ops ops, d4v (&acc)[T::FM][T::FN],
                              double* lds) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double ra[T::EA], rb[T::EB];
  unsigned za = 0u, zb = 0u;
  Opnd A, B;
  int k0;
  if (nsteps <= 0) return;
  auto fetch = [&](int s) {
    ops(s, A, B, k0);
    load_stage<T::BM, T::BK, T::EA, T::NT>(A, m0, k0, ra, za, tid);
    load_stage<T::BN, T::BK, T::EB, T::NT>(B, n0, k0, rb, zb, tid);
  };
  fetch(0);
  store_stage<T::BM, T::BK, T::EA, T::NT, T::LDA>(A.xfast, ra, za, lds, tid);
  store_stage<T::BN, T::BK, T::EB, T::NT, T::LDB>(B.xfast, rb, zb, lds + T::BK * T::LDA, tid);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    double* cur = lds + (s & 1) * T::STAGE;
    double* nxt = lds + ((s + 1) & 1) * T::STAGE;
    const bool more = (s + 1 < nsteps);
    if (more) fetch(s + 1);
    mfma_stage<T>(cur, cur + T::BK * T::LDA, acc, lane, wm, wn);
    if (more) {
      store_stage<T::BM, T::BK, T::EA, T::NT, T::LDA>(A.xfast, ra, za, nxt, tid);
      store_stage<T::BN, T::BK, T::EB, T::NT, T::LDB>(B.xfast, rb, zb, nxt + T::BK * T::LDA, tid);
    }
    __syncthreads();
  }
}

}  // namespace cc3
