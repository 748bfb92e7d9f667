// Two-centre metric kernels of all classes (L_P = 4, l_Q <= 4).
#include "registry.hpp"
namespace df3c {
void register_metric_lp4(MetricInfo (&t)[7]) { fill_metric<4>(t); }
}  // namespace df3c
