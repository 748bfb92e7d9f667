// Two-centre metric kernels of all classes (L_P = 2, l_Q <= 2).
#include "registry.hpp"
namespace df3c {
void register_metric_lp2(MetricInfo (&t)[7]) { fill_metric<2>(t); }
}  // namespace df3c
