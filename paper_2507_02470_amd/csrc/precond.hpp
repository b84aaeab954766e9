// precond.hpp -- interface of the diagonal preconditioning (precond.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Inputs: the given problem's explicit Q (CSR, NULL rowptr when Q = 0), A
// (CSR) and its stored A^T with the permutation at_perm[k] = position in A of
// entry k of A^T; the vectors c, L, U (n) and l, u (m).  All device pointers.
struct HqPrecondIn {
  int m, n;
  const int *a_rp, *a_ci; const double* a_v; int64_t a_nnz;
  const int *at_rp, *at_ci, *at_perm; const double* at_v;
  const int *q_rp, *q_ci; const double* q_v;
  const double *c, *L, *U, *l, *u;
  int ruiz_iters;
};

// Outputs (device, caller-allocated): scales D (n), E (m); scaled copies of
// the values of Q, A, A^T and of c, L, U, l, u; workspace of n, n and m doubles.
struct HqPrecondOut {
  double *D, *E;
  double *q_v, *a_v, *at_v;
  double *c, *L, *U, *l, *u;
  double *work_n, *work_n2, *work_m;
};

hipError_t hq_precondition(const HqPrecondIn& in, const HqPrecondOut& out, hipStream_t st);
