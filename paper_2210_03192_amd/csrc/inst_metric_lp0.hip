// Two-centre metric kernels of all classes (L_P = 0, l_Q <= 0).
#include "registry.hpp"
namespace df3c {
void register_metric_lp0(MetricInfo (&t)[7]) { fill_metric<0>(t); }
}  // namespace df3c
