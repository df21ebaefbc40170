// Host-side declarations of the transition-density loop (Algorithm 3): the
// kernel launchers of kern_density.hip and the loop itself.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cc3_internal.hpp"

namespace cc3 {

// One task of the Y^o / D_kc contractions: (cube index z in the batch, ordering
// index, p, q, r) for a distinct ordering (p, q, r) of an owned triple.
constexpr int D3_TASK_INTS = 5;

int d3_cd_chunks(int nv, int nown);
int d3_vec_chunks(int nv, int ntask, int ncol);
int d3_gram_chunks(int nv, int nz);
int d3_ld_chunks(int no, int nv);
size_t d3_partial_doubles(int no, int nv);

void launch_build_density_blocks(const CholeskyScratch& cs, double* Gw, double* Go, double* Jo,
                                 double* Go3, double* Gl, double* tmp, int no, int nv, int nJ,
                                 hipStream_t st);
void launch_d3_cd(const double* cubes, int64_t ss, const int* tri, int z0, int nown, double* P,
                  double* Dcd, int nv, hipStream_t st);
void launch_d3_vec(const double* cubes, int64_t ss, const int* task, int ntask, const double* t2,
                   const double* l2, double* Py, double* Pkc, double* Y, double* Dkc, int no,
                   int nv, hipStream_t st);
void launch_d3_gram(const double* cubes, int64_t ss, int z0, int nz, double* P, double* Dlk,
                    double scale, int no, int nv, hipStream_t st);
void launch_d3_ld(const double* Y, const double* t2, double* P, double* Dld, int no, int nv,
                  hipStream_t st);
void launch_d3_yout(const double* Y, double* Yo, int no, int nv, bool accumulate, hipStream_t st);
void launch_d3_l2m(const double* l2, double* l2M, int no, int nv, hipStream_t st);

}  // namespace cc3
