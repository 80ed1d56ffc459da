// Adjoint of the unrolled dual iteration (filled in with the backward pass).
#include "plan.h"
