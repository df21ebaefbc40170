// Device-side building blocks shared by the gfx950 kernels of libcc3: the
// FP64 MFMA tile engine (v_mfma_f64_16x16x4f64, 64-wide wavefronts, LDS-staged
// operands with register prefetch and double-buffered LDS).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc3 {

typedef double d4v __attribute__((ext_vector_type(4)));

// A strided 2D operand view: element (x, k) lives at p[x * sx + k * sk] and is
// multiplied by `scale`; outside [0, xlim) x [0, klim) it reads as zero.
// `xfast` selects the thread mapping used for the global loads: true when
// x is the contiguous index, false when k is.
struct Opnd {
  const double* p;
  int64_t sx, sk;
  int xlim, klim;
  double scale;
  bool xfast;
};

__device__ inline Opnd make_opnd(const double* p, int64_t sx, int64_t sk, int xlim, int klim,
                                 double scale, bool xfast) {
  Opnd o;
  o.p = p; o.sx = sx; o.sk = sk; o.xlim = xlim; o.klim = klim; o.scale = scale; o.xfast = xfast;
  return o;
}

// Tile geometry: WM x WN wavefronts, each owning FM x FN blocks of 16x16
// outputs; BK = 8 (two k=4 MFMA steps) per LDS stage.
template <int WM_, int WN_, int FM_, int FN_>
struct TileCfg {
  static constexpr int WM = WM_, WN = WN_, FM = FM_, FN = FN_;
  static constexpr int NW = WM * WN;
  static constexpr int NT = 64 * NW;
  static constexpr int BM = 16 * WM * FM;
  static constexpr int BN = 16 * WN * FN;
  static constexpr int BK = 8;
  static constexpr int LDA = BM + 16;  // row stride (doubles) of the k-major LDS tiles
  static constexpr int LDB = BN + 16;
  static constexpr int EA = (BM * BK + NT - 1) / NT;
  static constexpr int EB = (BN * BK + NT - 1) / NT;
  static constexpr int STAGE = BK * (LDA + LDB);  // doubles per LDS stage
  static constexpr int LDS_DOUBLES = 2 * STAGE;
};

// Global -> registers for one (X x BK) stage of an operand, x0/k0 the tile origin.
template <int X, int BK, int E, int NT>
__device__ inline void load_stage(const Opnd& o, int x0, int k0, double (&r)[E], int tid) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = e * NT + tid;
    int x, k;
    if (o.xfast) { x = idx % X; k = idx / X; } else { k = idx % BK; x = idx / BK; }
    double v = 0.0;
    if (idx < X * BK && x0 + x < o.xlim && k0 + k < o.klim)
      v = o.p[(int64_t)(x0 + x) * o.sx + (int64_t)(k0 + k) * o.sk] * o.scale;
    r[e] = v;
  }
}

// Registers -> k-major LDS tile s[k * LD + x] (same element mapping as load_stage).
template <int X, int BK, int E, int NT, int LD>
__device__ inline void store_stage(bool xfast, const double (&r)[E], double* s, int tid) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = e * NT + tid;
    if (idx < X * BK) {
      int x, k;
      if (xfast) { x = idx % X; k = idx / X; } else { k = idx % BK; x = idx / BK; }
      s[k * LD + x] = r[e];
    }
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
    double a[T::FM], b[T::FN];
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm) a[fm] = sa[kr * T::LDA + (wm * T::FM + fm) * 16 + (lane & 15)];
#pragma unroll
    for (int fn = 0; fn < T::FN; ++fn) b[fn] = sb[kr * T::LDB + (wn * T::FN + fn) * 16 + (lane & 15)];
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
// (k0 = first k of the step within its operands); `after(step)` runs after the
// MFMAs of each step (used to flush partial results).  Double-buffered LDS with
// one barrier per step; the next stage's global loads are in flight during the
// current stage's MFMAs.
template <class T, class Ops, class After>
__device__ inline void k_loop(int nsteps, int m0, int n0, Ops ops, After after,
                              d4v (&acc)[T::FM][T::FN], double* lds) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % T::WM, wn = wave / T::WM;
  double ra[T::EA], rb[T::EB];
  Opnd A, B;
  int k0;
  if (nsteps <= 0) return;
  ops(0, A, B, k0);
  load_stage<T::BM, T::BK, T::EA, T::NT>(A, m0, k0, ra, tid);
  load_stage<T::BN, T::BK, T::EB, T::NT>(B, n0, k0, rb, tid);
  store_stage<T::BM, T::BK, T::EA, T::NT, T::LDA>(A.xfast, ra, lds, tid);
  store_stage<T::BN, T::BK, T::EB, T::NT, T::LDB>(B.xfast, rb, lds + T::BK * T::LDA, tid);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    double* cur = lds + (s & 1) * T::STAGE;
    double* nxt = lds + ((s + 1) & 1) * T::STAGE;
    const bool more = (s + 1 < nsteps);
    if (more) {
      ops(s + 1, A, B, k0);
      load_stage<T::BM, T::BK, T::EA, T::NT>(A, m0, k0, ra, tid);
      load_stage<T::BN, T::BK, T::EB, T::NT>(B, n0, k0, rb, tid);
    }
    mfma_stage<T>(cur, cur + T::BK * T::LDA, acc, lane, wm, wn);
    after(s);
    if (more) {
      store_stage<T::BM, T::BK, T::EA, T::NT, T::LDA>(A.xfast, ra, nxt, tid);
      store_stage<T::BN, T::BK, T::EB, T::NT, T::LDB>(B.xfast, rb, nxt + T::BK * T::LDA, tid);
    }
    __syncthreads();
  }
}

}  // namespace cc3
