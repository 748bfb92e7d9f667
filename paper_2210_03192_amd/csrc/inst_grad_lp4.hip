// Backward (J-gradient) kernels of all classes with an auxiliary shell of
// l = 4 (one translation unit per l so the build parallelises).
#include "registry.hpp"
DF3C_REGISTER_GRAD_LP(4, register_grad_lp4)
