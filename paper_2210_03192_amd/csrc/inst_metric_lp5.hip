// Two-centre metric kernels of all classes (L_P = 5, l_Q <= 5).
#include "registry.hpp"
namespace df3c {
void register_metric_lp5(MetricInfo (&t)[7]) { fill_metric<5>(t); }
}  // namespace df3c
