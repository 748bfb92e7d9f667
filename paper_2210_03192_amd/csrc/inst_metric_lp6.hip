// Two-centre metric kernels of all classes (L_P = 6, l_Q <= 6).
#include "registry.hpp"
namespace df3c {
void register_metric_lp6(MetricInfo (&t)[7]) { fill_metric<6>(t); }
}  // namespace df3c
