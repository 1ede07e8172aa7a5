// The kernels of the factorization chain as one translation unit: the sketch, the
// tall-skinny solve and Gram, the small factorizations, the low-precision phases, and the
// persistent batched kernel that runs all of their device bodies in one launch.  The
// included files are not compiled on their own.
#include "k_sketch.hip"
#include "k_tall.hip"
#include "k_small.hip"
#include "k_lowp.hip"
#include "k_persist.hip"
