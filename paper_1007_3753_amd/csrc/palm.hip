// PALM driver kernels (filled in with the primal method).
#include "plan.h"
