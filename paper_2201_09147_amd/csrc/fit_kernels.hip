// fit_kernels.hip -- placeholder until the fitting kernels land.
#include "nnm_kernels.h"
