// Discrete adjoint of the time step (written in the next revision).
#include "fvib_kernels.h"

extern "C" int fvib_step_adjoint(fvib_grid*, const fvib_fields*, const fvib_adjoint*,
                                 const double*, fvib_adjoint*, fvib_step_info*) {
  return FVIB_ESTATE;
}
