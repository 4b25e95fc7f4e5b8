// Backward (adjoint) kernels of the ray-wave hybrid PSF.
#pragma once
#include "rw_kernels.h"

#define RW_LENSG_SLOTS 128

struct rw_plan;
static rw_status rw_backward_impl(rw_plan* pl, const float* dL_dpsf, float* d_phase, float* d_amp,
                                  float* d_lens, void* ws, size_t ws_bytes, void* stream);
