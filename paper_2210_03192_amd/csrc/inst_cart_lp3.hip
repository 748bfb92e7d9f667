// Store kernels with a Cartesian ket for the classes with an auxiliary shell
// of l = 3 (aux pure = 0; one translation unit per l).
#include "registry.hpp"
DF3C_REGISTER_CART_LP(3, register_cart_lp3)
