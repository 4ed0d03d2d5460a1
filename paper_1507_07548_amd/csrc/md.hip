// Device-resident MD step kernels (filled in with the batched path).
#include <hip/hip_runtime.h>

#include "internal.h"
