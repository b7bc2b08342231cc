// The kernels of the iteration for two-word determinants (65 to 128 spin orbitals),
// compiled from the same source into namespace fq::w2.
#define FQ_DET_WORDS 2
#include "kernels.hip"
