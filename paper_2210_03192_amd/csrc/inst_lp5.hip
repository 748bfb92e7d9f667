// Kernels of all classes with an auxiliary shell of l = 5 (one translation
// unit per l so the build parallelises).
#include "registry.hpp"
DF3C_REGISTER_LP(5, register_lp5)
