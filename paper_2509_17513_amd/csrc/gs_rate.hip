// Rate model of the quantised Gaussian attributes (filled in below).
#include <hip/hip_runtime.h>

#include "gs4d.h"
