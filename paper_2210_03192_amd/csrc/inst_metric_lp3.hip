// Two-centre metric kernels of all classes (L_P = 3, l_Q <= 3).
#include "registry.hpp"
namespace df3c {
void register_metric_lp3(MetricInfo (&t)[7]) { fill_metric<3>(t); }
}  // namespace df3c
