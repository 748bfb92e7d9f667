// Two-centre metric kernels of all classes (L_P = 1, l_Q <= 1).
#include "registry.hpp"
namespace df3c {
void register_metric_lp1(MetricInfo (&t)[7]) { fill_metric<1>(t); }
}  // namespace df3c
