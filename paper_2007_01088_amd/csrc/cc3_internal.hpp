// Host-side declarations shared by the host core (cc3_core.cpp) and the kernel
// translation units: the workspace plan and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cc3 {

// Most triples per batch of the triple loop.  A batch holds at most two
// (triple, permutation) pairs per triple with a given first occupied index, so
// the per-p pair lists of the kernels hold 2 * MAX_BATCH entries.
constexpr int MAX_BATCH = 160;

// Internal plan flag (beside the public CC3_* flags): the triple loop runs every
// batch on the caller's stream and records no events (the allocation-free entry point).
constexpr unsigned PLAN_CALLER_STREAM = 1u << 30;

// triple kinds
enum { TRI_DISTINCT = 0, TRI_IJ = 1, TRI_JK = 2 };

// The kind of an ordered triple for the W build and mix: equal neighbours in the
// first two or the last two positions let three of the six P terms repeat.  An
// all-equal triple (which the residual's loop skips; the transition-density loop
// needs its t3) takes every term.
__host__ __device__ inline int tri_kind(int i, int j, int k) {
  if (i == j && j == k) return TRI_DISTINCT;
  if (i == j) return TRI_IJ;  // i == j, k different
  if (j == k) return TRI_JK;  // j == k, i different
  return TRI_DISTINCT;
}

// The occupied permutation pi of (i,j,k) used for the contravariant contributions:
// 0 (i,j,k)  1 (j,i,k)  2 (k,j,i)  3 (i,k,j)  4 (j,k,i)  5 (k,i,j).
// All six are distinct when i, j, k differ; {0,2,3} when i == j; {0,1,2} when j == k.
__host__ __device__ inline bool perm_active(int kind, int pi) {
  if (kind == TRI_IJ) return pi == 0 || pi == 2 || pi == 3;
  if (kind == TRI_JK) return pi <= 2;
  return true;
}

__host__ __device__ inline void perm_pqr(int pi, int i, int j, int k, int& p, int& q, int& r) {
  switch (pi) {
    case 0: p = i; q = j; r = k; break;
    case 1: p = j; q = i; r = k; break;
    case 2: p = k; q = j; r = i; break;
    case 3: p = i; q = k; r = j; break;
    case 4: p = j; q = k; r = i; break;
    default: p = k; q = i; r = j; break;
  }
}

// K padded to a multiple of 32 (the low-precision operand rows)
__host__ __device__ inline int64_t kpad32(int64_t k) { return (k + 31) / 32 * 32; }

// K of the split-BF16 Omega contraction (the mixed-all form): the pair (x, y) of the
// contracted virtual indices in 8 x 8 blocks, kb = ((X nb + Y) 8 + x % 8) 8 + y % 8 with
// X = x / 8, Y = y / 8 and nb = ceil(nv / 8), so that the 64 values of one block, which
// the mix holds together, are contiguous; positions with x or y >= nv hold zeros.
__host__ __device__ inline int64_t lp_kb_len(int nv) {
  const int64_t nb = (nv + 7) / 8;
  return nb * nb * 64;
}
// Row pitch of those operands: Kb plus 32 values, so that rows do not fall a power of
// two apart (Kb is one whenever nv / 8 is) and share memory channels.
__host__ __device__ inline int64_t lp_kb_pitch(int nv) { return lp_kb_len(nv) + 32; }
__host__ __device__ inline int64_t lp_kb(int x, int y, int nv) {
  const int nb = (nv + 7) / 8;
  return ((int64_t)((x >> 3) * nb + (y >> 3)) * 8 + (x & 7)) * 8 + (y & 7);
}

// The cubes of the triple loop (W planes P0..P2, tau~ and tau~T, [x][y][z] per slot)
// keep their rows of nv values at a pitch padded to a multiple of 8 doubles, so that the
// row segments of 8 or 16 values that the W build, the mix and the Omega kernels move
// start on 64-byte boundaries; the padding columns are never read.  cube_slot is the
// doubles of one slot.  (The low-precision copies and the transition-density cubes
// are not padded.)
__host__ __device__ inline int cube_pitch(int nv) { return (nv + 7) & ~7; }
__host__ __device__ inline int64_t cube_slot(int nv) {
  return (int64_t)nv * nv * cube_pitch(nv);
}

// Device-resident, internally laid out integral blocks (all float64):
//   Gw[r][y][z][d] = g_{ydzr}         (vv|vo), the W contraction operand (d fastest)
//   Go[q][r][z][l] = g_{lqzr}         (oo|vo) (l fastest)
//   Gbc[r][n][b][c] = g_{nbrc} for n < nv (vv|ov), g_{lbrc} for n = nv + l (ov|ov):
//                     the Omega contraction operand, K = (b, c) contiguous
//   Gcb[r][n][c][b] = the same values with K = (c, b) contiguous
//   Jo[q][r][b][c] = g_{qbrc}         (ov|ov)
//   Hs[q][r][c][l] = delta_{lq} F_rc - g_{qlrc}   (oo|ov) and the Fock ov block (l fastest)
//   F[k][c]
struct Blocks {
  double* Gw;
  double* Go;
  double* Gbc;
  double* Gcb;
  double* Jo;
  double* Hs;
  double* F;
};

// Intermediates of the T1 transformation (Cholesky form only):
//   Lvv[J][b][d] = Lt_{bd}, Loo[J][q][l] = Lt_{ql},
//   LooT[J][l][q] = Lt_{ql}, LvoT[J][k][c] = Lt_{ck}, Lov[J][k][c] = L_{kc},
//   s[J], M[J][k][l]: partial sums of the Fock ov block.
struct CholeskyScratch {
  double *Lvv, *Loo, *LooT, *LvoT, *Lov, *s, *M;
};

struct Plan {
  int no, nv, nchol, prec;
  unsigned flags;
  int ntri;     // unordered triples i >= j >= k, not all equal
  int batch;    // triples per batch of the triple loop
  size_t pvv_entries;  // max (triples x chunks) of one Omega or Zo launch
  size_t cube;  // doubles per cube slot (cube_slot: nv x nv rows at the padded pitch)
  // byte offsets into the workspace
  size_t off_blocks;  // integral blocks (when the workspace holds them)
  size_t off_Ot1, off_Ot2, off_OtT, off_lp, off_t2N, off_Pvv, off_tri, off_flag, off_cubes;
  size_t off_gf, gf_bytes;        // mixed-all: low-precision Gbc and Gcb (0 bytes otherwise)
  size_t off_cubef, cubef_bytes;  // mixed-all: low-precision views of tau~, per buffer set
  size_t off_chol;  // Cholesky scratch (aliases the cube region)
  // one-shot calls only (0 otherwise): staging of host-memory arguments, eps, t1, t2
  // and omega1 at off_stage; a host L, or the host integral blocks, pass through
  // the cube region during setup (stage_region bytes from off_cubes)
  size_t off_stage, stage_region;
  size_t chol_bytes, cube_bytes, pvv_bytes;  // per buffer set (two sets)
  size_t total;
};

// Low-precision copies of the W operands (FP32, or BF16 pieces), see kern_wlp.hip.
struct LpOperands {
  void *t2, *t2N, *GwT, *GoT;
  int prec;
};
size_t lp_operand_bytes(int prec, int no, int nv);
void lp_operand_ptrs(int prec, int no, int nv, void* base, LpOperands& lp);
void launch_lp_convert(const double* t2, const Blocks& b, int no, int nv, const LpOperands& lp,
                       hipStream_t st);
void launch_wbuild_lp(const LpOperands& lp, const int* tri, int ntri, double* cubes, int no, int nv,
                      bool all_terms, hipStream_t st);

// ---- launchers (all enqueue on `st`) ----
void launch_fill(double* p, int64_t n, double v, hipStream_t st);
void launch_add(double* y, const double* x, int64_t n, hipStream_t st);  // y += x
void launch_t1_transform(const double* L, const double* t1, const CholeskyScratch& cs, int no,
                         int nv, int nJ, hipStream_t st);
void launch_fock(const double* t1, const CholeskyScratch& cs, double* F, int no, int nv, int nJ,
                 hipStream_t st);
void launch_build_blocks(const CholeskyScratch& cs, const Blocks& b, int no, int nv, int nJ,
                         hipStream_t st);
// The paper-order blocks into the internal layouts, in three parts: the
// (oo|vo), (ov|ov), (oo|ov) and Fock blocks; the (vv|vo) and (vv|ov) blocks for
// the first virtual index y in [y0, y0 + ny), read from g_vvvo_y = &g_vvvo[y0][0][0][0]
// and g_vvov_y = &g_vvov[y0][0][0][0]; then the (c, b) copy of Gbc (launch_gcb).
void launch_relayout_small(const double* g_oovo, const double* g_ovov, const double* g_ooov,
                           const double* F_ov, const Blocks& b, int no, int nv, hipStream_t st);
void launch_relayout_vv(const double* g_vvvo_y, const double* g_vvov_y, int y0, int ny,
                        const Blocks& b, int no, int nv, hipStream_t st);
void launch_gcb(const Blocks& b, int no, int nv, hipStream_t st);
// The full triple table, the restricted loop dealt round-robin over nbatch batches.
void launch_triple_table(int* tri, int no, int nbatch, hipStream_t st);
void launch_t2N(const double* t2, double* t2N, int no, int nv, hipStream_t st);
void launch_wbuild(const double* t2, const double* t2N, const Blocks& b, const int* tri, int ntri,
                   double* cubes, int no, int nv, bool all_terms, hipStream_t st);
// The W build's engine with explicit operands and output strides (doubles between
// triples, zs, between the three planes, ss, and between the rows of a plane, pitch).
// mode 0: the t3 terms (X = t2, XN = t2N, G = Gw, H = Go); mode 1: the left-state L3
// terms of Algorithm 3 without their outer-product parts (X = l2, XN = l2M, G = Gl,
// H = Go3).
void launch_wbuild_ex(int mode, const double* X, const double* XN, const double* G, const double* H,
                      const int* tri, int ntri, double* cubes, int64_t zs, int64_t ss, int pitch,
                      int no, int nv, bool all_terms, hipStream_t st);
// Mixed-all copies (nullable): cubesF, FP32 tau~ and tau~T, [triple][2][nv^3]; YL,
// the split-BF16 k-major views of k_omega_lp with lpP pieces
void launch_mix(const double* eps, const int* tri, int ntri, double* cubes, float* cubesF,
                void* YL, int lpP, int no, int nv, hipStream_t st);
void launch_tau_export(const double* eps, const int* tri, const double* cubes, double* tau, int no,
                       int nv, hipStream_t st);
// Omega contraction of a batch: the vv term and Omega1 into per-(triple,
// permutation, chunk) partial slabs Pvv, then their fixed-order reduction into
// Ot1/Ot2 (added, not overwritten); the oo and Fock terms added into OtT
// (output-stationary).  The reduction and the OtT update of successive batches
// must run in batch order.
void launch_omega(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Pvv,
                  int no, int nv, hipStream_t st);
void launch_reduce(const int* tri, int ntri, const double* Pvv, double* Ot1, double* Ot2, int no,
                   int nv, bool fp32acc, hipStream_t st);
void launch_omega_oo(const double* cubes, const Blocks& b, const int* tri, int ntri, double* OtT,
                     int no, int nv, hipStream_t st);
// The mixed-all form of launch_omega: FP32 MFMA over FP32 copies of the cubes
// (tau~, tau~T per triple) and of Gbc / Gcb; partial slabs in FP64 as above.
void launch_omega_f32(const float* cubesF, const float* GbcF, const float* GcbF, const int* tri,
                      int ntri, double* Pvv, int no, int nv, hipStream_t st);
void launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st);
// The mixed-all form with split BF16 (kern_wlp.hip): bytes of one of the two
// operand blocks and of one triple's views; their conversion, the views' K
// padding, and the GEMM.
size_t lp_contract_g_bytes(int prec, int no, int nv);
size_t lp_contract_cube_bytes(int prec, int nv);
void launch_lp_contract_convert(const Blocks& b, int prec, int no, int nv, void* GbcL, void* GcbL,
                                hipStream_t st);
void launch_lp_zero_pad(void* YL, int64_t rows, int nv, hipStream_t st);
void launch_omega_lp(int prec, const void* YL, const void* GbcL, const void* GcbL, const int* tri,
                     int ntri, double* Pvv, int no, int nv, hipStream_t st);
// Ot~2[p][q][a][b] = Ot2[p][q][a][b] + OtT[p][q][b][a]  (contravariant doubles residual)
void launch_combine(const double* Ot1, const double* Ot2, const double* OtT, double* O1,
                    double* O2, int no, int nv, hipStream_t st);
// K chunks of one Omega GEMM; fp32acc: its chunks are summed in FP32 (the mixed-all
// forms), at most 4096 k each
int omega_kchunks(int nv, int ntri, bool fp32acc = false);
int zo_nbchunks(int nv, int ntri);    // b chunks of one Zo product
void launch_back_transform(const double* Ot1, const double* Ot2, const double* OtT, double* O1,
                           double* O2, int no, int nv, bool accumulate, hipStream_t st);
void launch_set_triples(int* tri_dev, const int* host_tri, int n, hipStream_t st);
void launch_check(const double* eps, const double* L, const double* t2, int no, int nv, int nJ,
                  int* flag, hipStream_t st);

// Preparation for the Jacobian transformations (Algorithm 2), per batch:
// Zv -= (read-modify-write, output-stationary); Zo partials into Pzo (reduce = false),
// then their fixed-order sum into Zo (reduce = true).
void launch_zv(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Zv, int no,
               int nv, hipStream_t st);
void launch_zo(const double* cubes, const Blocks& b, const int* tri, int ntri, double* Pzo,
               double* Zo, int no, int nv, hipStream_t st, bool reduce);
double zprep_flops(int no, int nv, const int* host_types, int n);

// ---- packing small serving requests into shared persistent launches ----
// One packed launch runs one kernel of the triple loop (W build, mix, Omega,
// oo, reduction) for the current batch of several requests: its workgroups loop
// over the union of the jobs' work items, each item taking the job's operands.
enum { PK_W = 0, PK_MIX, PK_OMEGA, PK_OO, PK_RED, PK_N };
struct PackJob {
  const double *t2, *t2N, *eps;
  const double *Gw, *Go, *Gbc, *Gcb, *Hs;
  const void *lpt2, *lpt2N, *lpGwT, *lpGoT;  // low-precision W operands (FP32, split BF16)
  const int* tri;                             // the job's batch of triples
  double *cubes, *Pvv, *Ot1, *Ot2, *OtT;
  int no, nv, ntri, nch;
  unsigned first[PK_N];  // first packed work item of this job, per kernel
};
// Work items of one job per kernel (the workgroups of its unpacked launch).
void pack_items(const PackJob& j, unsigned (&items)[PK_N]);
// The five packed launches of one step (jobs in device memory, host copy for the
// item counts); prec: the W build's arithmetic, shared by every job.
void launch_packed_step(const PackJob* dev_jobs, const PackJob* host_jobs, int njobs, int prec,
                        hipStream_t st);

// ---- transition densities (Algorithm 3) ----
// Slots of the density loop's cubes, slot-major: cubes[slot][z][cube_slot(nv)].
enum { D3_P0 = 0, D3_P1 = 1, D3_P2 = 2, D3_TAU = 3, D3_TAUC = 4, D3_LC = 5, D3_NSLOT = 6 };
// tau, tau~ (lmode false) or L~ (lmode true, with the outer products of the L3
// statement from l1, l2, Jo, F and the shift omega) from the planes of each triple
void launch_mix3(bool lmode, const double* eps, const int* tri, int ntri, double* cubes, int64_t ss,
                 double omega, const double* l1, const double* l2, const double* Jo,
                 const double* F, int no, int nv, hipStream_t st);

// Algorithmic FLOP of one launch of the two dominant kernels (padding excluded).
double wbuild_flops(int no, int nv, const int* host_types, int n);
double omega_flops(int no, int nv, const int* host_types, int n);
double omega_oo_flops(int no, int nv, const int* host_types, int n);

}  // namespace cc3
