/* Surrogate network of the parameter sweep: a 4 -> 128 -> 128 -> 2
 * multilayer perceptron (SiLU hidden layers, sigmoid outputs) that maps
 * normalised sweep parameters to the equilibrium bonded fraction and
 * largest-cluster fraction measured by the simulator, trained on the GPU with
 * mean-squared error and Adam.
 *
 * Precision: the FP32 master weights are rounded to bfloat16 for every
 * layer; the 128 x 128 layer and both GEMMs of its backward pass run on the
 * matrix cores (bf16 inputs, FP32 accumulation) with the hidden activation
 * a1 and the back-propagated dz2 rounded to bf16; biases, the other
 * activations, gradients and Adam state are FP32.
 *
 * Parameters are one flat FP32 vector: W1 (128 x 4, row-major), b1 (128),
 * W2 (128 x 128), b2 (128), W3 (2 x 128), b3 (2); DB_MLP_PARAMS numbers.
 * Inputs are n x 4 and targets / outputs n x 2 row-major FP32 host arrays,
 * borrowed for the call.  Every call is synchronous.  A handle is not
 * thread-safe.  Errors are returned as db_status (dybond.h); the message is
 * in db_mlp_last_error.
 */
#ifndef DYBOND_MLP_H
#define DYBOND_MLP_H

#include "dybond.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DB_MLP_PARAMS 17410u

typedef struct db_mlp db_mlp;

/* Network on HIP device `device` for minibatches of up to batch_max rows
 * (1..4096; rounded up internally to a multiple of 16).  Parameters start at
 * zero; set them with db_mlp_set_params.  Errors: DB_EINVAL, DB_EDEVICE,
 * DB_ENOMEM. */
DB_API db_status db_mlp_create(uint32_t batch_max, int device, db_mlp** out);

/* Free the device buffers and the handle (NULL is a no-op). */
DB_API void db_mlp_destroy(db_mlp* net);

/* Copy `count` (== DB_MLP_PARAMS) FP32 parameters in; resets Adam's moments
 * and step count.  Errors: DB_EINVAL. */
DB_API db_status db_mlp_set_params(db_mlp* net, const float* params, uint64_t count);

/* Copy the FP32 master parameters out (count == DB_MLP_PARAMS). */
DB_API db_status db_mlp_get_params(db_mlp* net, float* params, uint64_t count);

/* Outputs y (n x 2) for inputs x (n x 4), any n (processed batch_max rows
 * at a time). */
DB_API db_status db_mlp_predict(db_mlp* net, const float* x, uint64_t n, float* y);

/* Mean-squared error of the outputs against targets t over n rows
 * (1 <= n <= batch_max) and its gradient with respect to the FP32
 * parameters (DB_MLP_PARAMS floats into grad), computed by the device's
 * forward and backward passes; parameters are not changed. */
DB_API db_status db_mlp_loss_grad(db_mlp* net, const float* x, const float* t, uint32_t n, float* loss,
                                  float* grad);

/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) for
 * `epochs` passes over the n rows, in minibatches of `batch` rows
 * (1..batch_max; the last one of an epoch may be smaller) drawn in a fresh
 * order every epoch from a generator seeded with `seed`.  *final_loss (may
 * be NULL) receives the mean-squared error over all n rows after training.
 * The Adam step count continues across calls.  Errors: DB_EINVAL. */
DB_API db_status db_mlp_train(db_mlp* net, const float* x, const float* t, uint64_t n, uint32_t batch,
                              uint32_t epochs, float lr, uint64_t seed, float* final_loss);

/* Last error message of this handle ("" if none). */
DB_API const char* db_mlp_last_error(const db_mlp* net);

#ifdef __cplusplus
}
#endif

#endif
