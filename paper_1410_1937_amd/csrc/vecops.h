// Launchers of the solver vector kernels (vecops.hip).
#pragma once

#include "nfa_internal.h"

namespace nfa {

// finalize phases: what a reduction feeds into the solver state
enum { PH_BB = 0, PH_RR = 1, PH_INIT = 2, PH_PQ = 3, PH_UPD = 4, PH_RRO = 5, PH_ZQ = 6, PH_PR = 7,
       PH_PQF = 8, PH_UPDF = 9, PH_RELIABLE = 10, PH_RELIABLE_F = 11, PH_PQ_SKIP = 12 };

void launch_finalize(const double* partials, int n, int ncomp, int phase, SolveScalars* sc,
                     double* hist, hipStream_t s);
// launch_finalize together with a merge gather (gather) or copy of v
template <class T>
void launch_finalize_merge(const Grid& g, bool gather, T* v, const double* partials, int n, int ncomp,
                           int phase, SolveScalars* sc, double* hist, hipStream_t s);
template <class T> int launch_dot(const T* a, const T* b, long long n, double* partials,
                                  const SolveScalars* sc, hipStream_t s);
template <class T> int launch_masked_sum(const T* a, const unsigned char* mask, long long n,
                                         double* partials, hipStream_t s);
void launch_sub_mean(double* b, const unsigned char* mask, long long n, const double* sum,
                     double count, hipStream_t s);
template <class T> int launch_jacobi(const T* r, const T* dinv, T* z, long long n, double* partials,
                                     hipStream_t s);
template <class T> void launch_copy(const T* a, T* b, long long n, hipStream_t s);
template <class T> void launch_fill(T* a, T v, long long n, hipStream_t s);
void launch_init_x(double* x, const unsigned char* act, long long n, int warm, hipStream_t s);
void launch_set_scalars(SolveScalars* sc, double t, int tol_mode, int max_iter, int reset_iter,
                        int window, double ratio, hipStream_t s);
template <class T> void launch_scale(const T* r, const T* dinv, T* z, long long n, const SolveScalars* sc,
                                     hipStream_t s);
template <class T> void launch_sabotage(const unsigned char* red, T* z, long long n, const SolveScalars* sc,
                                        hipStream_t s);

// fused CG sweeps (cg.hip)
template <class T> bool cg_vectorizable(const Grid& g, const void* const* ptrs, int nptr);
template <class T>
int launch_cg_a(const Grid& g, const Coeffs<T>& C, const T* z, const T* pold, const T* pold2, T* pnew,
                T* x, const T* r, T* q, double* partials, const SolveScalars* sc, bool flex, int xm,
                bool vec, hipStream_t s);
template <class T>
int launch_cg_b(const Grid& g, T* r, const T* q, const T* dinv, T* z, double* partials,
                const SolveScalars* sc, bool flex, bool vec, hipStream_t s);
template <class T>
void launch_cg_fixup(const Grid& g, T* x, const T* p, const T* p2, const SolveScalars* sc, hipStream_t s);
void launch_fold(const Grid& g, double* x, float* d, double inv_scale, hipStream_t s);
void launch_cast(const Grid& g, const double* r, float* r32, double scale, hipStream_t s);

}  // namespace nfa
