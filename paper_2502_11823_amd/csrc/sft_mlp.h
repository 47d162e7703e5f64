// sft_mlp.h -- internal interface of the surrogate network engine (libsft.so only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sft.h"

// The network: u (3) -> [W_l, b_l, SiLU] x layers (width hidden) -> W_out, b_out -> y (2).
// Parameters packed layer by layer: W [n_in][n_out] (input-major), then b [n_out].
struct sft_surrogate {
  sft_surrogate_desc d;
  int64_t P;          // parameter count
  float* par;         // [P] FP32 parameters (trained)
  float* grad;        // [P]
  float* mom1;        // [P] Adam first moment
  float* mom2;        // [P] Adam second moment
  double* par_inf;    // [P] inference copy: FP64 values of the FP32 (or BF16-rounded) parameters
  void* frag;         // BF16 inference: the hidden-to-hidden weights as packed MFMA fragments (or null)
  int32_t step;       // Adam step count
  int device;
};

// record msg as the thread's last error (sft_last_error) and return st
sft_status sft_set_error(sft_status st, const char* msg);

struct MlpLayer {
  int n_in, n_out;
  int64_t w_off, b_off;
};

// geometry of layer l (0..layers; the last one is the output layer)
MlpLayer mlp_layer(int hidden, int layers, int l);
int64_t mlp_param_count(int hidden, int layers);

// scratch needed by mlp_infer for chunks of `chunk` rows
size_t mlp_infer_scratch_bytes(int hidden, int64_t chunk);

// FP64 forward pass with the forward-mode derivative along input 3 for n rows of U
// ([n][3], row-major): Y [n][2], dY [n][2].  Uses the FP64 inference copy of the
// parameters; scratch holds mlp_infer_scratch_bytes(hidden, min(n, chunk)) bytes.
hipError_t mlp_infer(const sft_surrogate* s, const double* U, int64_t n, double* Y, double* dY, void* scratch,
                     int64_t chunk, hipStream_t st);
