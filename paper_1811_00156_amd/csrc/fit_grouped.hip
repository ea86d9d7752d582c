// The grow kernels of fused fits that grow task groups (trees of forests that
// differ only in min.node.size, grown together down to the level where they
// part): the kernel templates of fit.hip instantiated with groups, in a
// translation unit of their own so that they compile alongside the others.
#define AIWC_GROW_GROUPED 1
#include "fit.hip"
