// Backward (J-gradient) kernels of all classes with an auxiliary shell of
// l = 1 (one translation unit per l so the build parallelises).
#include "registry.hpp"
DF3C_REGISTER_GRAD_LP(1, register_grad_lp1)
