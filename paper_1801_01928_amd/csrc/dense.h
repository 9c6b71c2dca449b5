// Dense sweeps of the Riemannian step (dense.hip).
#pragma once
#include "common.h"

namespace ttgfx {

#define DENSE_MAX_RANK 64

int dense_orth_ranks(const tt_tensor *X, int dir, int32_t *out);
int dense_round_ranks(const tt_tensor *Y, int max_rank, int32_t *out);
size_t dense_ws(const tt_tensor *X);
int dense_orth(const tt_tensor *X, int dir, tt_tensor *O, void *ws, size_t bytes, hipStream_t s);
int dense_orth_both(const tt_tensor *X, tt_tensor *OL, tt_tensor *OR, void *ws, size_t bytes, hipStream_t s);
int dense_round(const tt_tensor *Y, int max_rank, tt_tensor *O, float *disc, int *status, void *ws, size_t bytes,
                hipStream_t s);
size_t tangent_ws(const tt_tensor *U);
size_t project_tt_ws(const tt_tensor *U, const tt_tensor *Y);
int project_tt(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Y, float alpha, int add_x, tt_tensor *W,
               void *ws, size_t bytes, hipStream_t s);
int tangent_combine(const tt_tensor *U, const tt_tensor *P, tt_tensor *W, float alpha, int add_x,
                    hipStream_t s);
size_t project_sum_ws(const tt_tensor *U, const tt_tensor *A0, int nb);
int project_sum(const tt_tensor *U, const tt_tensor *V, const tt_tensor *A, int nb, const float *c, float alpha,
                int add_x, tt_tensor *W, void *ws, size_t bytes, hipStream_t s);
int tangent_combine_dev(const tt_tensor *U, const tt_tensor *P, tt_tensor *W, const float *alpha, float scale,
                        int add_x, hipStream_t s);
// One direction update of nonlinear CG (txi = teta = NULL on the first step);
// sc: (dev) float [5] scalars (see cg_beta_kernel).
int cg_direction(const tt_tensor *U, const tt_tensor *xi, const tt_tensor *txi, const tt_tensor *teta,
                 const float *prev_sq, tt_tensor *eta, float *sc, hipStream_t s);
int tangent_inner(const tt_tensor *U, const tt_tensor *A, const tt_tensor *B, float *out, hipStream_t s);
int tangent_axpby(const tt_tensor *U, float a, const tt_tensor *A, float b, const tt_tensor *B, tt_tensor *W,
                  hipStream_t s);
size_t tangent_gram_ws(const tt_tensor *U, int nb);
int tangent_gram(const tt_tensor *U, const tt_tensor *A, int nb, float *G, void *ws, size_t bytes, hipStream_t s);
int tangent_assemble(const tt_tensor *U, const tt_tensor *V, const tt_tensor *Z, tt_tensor *W,
                     float alpha, int add_x, void *ws, size_t bytes, hipStream_t s);

}  // namespace ttgfx
