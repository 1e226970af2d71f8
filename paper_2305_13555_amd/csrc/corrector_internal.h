// Entry points of the corrector (corrector.hip) that the OCI driver uses to
// apply a corrector inside the iteration (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "oci.h"

// y [4][cells] = f(x [8][cells]) in FP32 on the matrix cores, enqueued on st;
// OCI_EINVAL for NULL pointers or cells outside [1, the corrector's maximum].
int occ_infer32(oci_corrector *k, hipStream_t st, const float *x, int cells, float *y);
// The corrector's channel counts and the most cells one inference takes.
int occ_channels(const oci_corrector *k, int *c_in, int *c_out, int64_t *max_cells);
