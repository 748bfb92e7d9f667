// Per-class launch configuration and the launcher table shared by the
// instantiation units and the runtime.
#pragma once
#include "gamma.hpp"
#include "grad.hpp"
#include "metric.hpp"
#include "queue.hpp"

namespace df3c {

struct ClassInfo {
  int ts = 0;         // lanes per team
  int tpw = 0;        // teams per workgroup (block kernels)
  int tpwj = 0;       // teams per workgroup of the J kernels
  int jreg = 0;       // J on the register engine (one lane, or nsub lanes, per pair)
  int lds = 0;        // dynamic LDS bytes per workgroup
  hipError_t (*store)(const StoreArgs &, int, hipStream_t) = nullptr;
  // Cartesian-ket instantiation (aux pure = 0; the same kernel for l <= 1)
  hipError_t (*store_cart)(const StoreArgs &, int, hipStream_t) = nullptr;
  hipError_t (*jfn)(const JArgs &, int, hipStream_t) = nullptr;
  hipError_t (*jq)(const JQArgs &, int, hipStream_t) = nullptr;
  hipError_t (*gam)(const GamArgs &, int, hipStream_t) = nullptr;
};

struct MetricInfo {
  int ppw = 0;        // shell pairs per workgroup and grid step
  hipError_t (*fn)(const MetArgs &, int, hipStream_t) = nullptr;
};

struct GradInfo {
  int tpb = 0;        // per-atom LDS arrays (teams) per workgroup
  int team = 0;       // LDS doubles per team before the per-atom array
  int ppw = 0;        // shell pairs per workgroup and grid step
  int wpb = 0;        // wavefronts per workgroup
  int min_aux = 1;    // fewest aux shells per work item worth the per-pair set-up
  hipError_t (*gfn)(const GradArgs &, int, int, hipStream_t) = nullptr;  // (args, grid, lds)
};

template <int LP, int LA, int LB>
hipError_t launch_store(const StoreArgs &a, int grid, hipStream_t s) {
  using C = Cfg<LP, LA, LB>;
  auto kern = k_store<LP, LA, LB, C::TS, C::PCH>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
      C::STORE_LDS_V);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::BLK), C::STORE_LDS_V, s, a);
  return hipGetLastError();
}

template <int LP, int LA, int LB>
hipError_t launch_store_cart(const StoreArgs &a, int grid, hipStream_t s) {
  using C = Cfg<LP, LA, LB>;
  auto kern = k_store<LP, LA, LB, C::TS, C::PCH, true>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
      C::STORE_LDS_CV);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::BLK), C::STORE_LDS_CV, s, a);
  return hipGetLastError();
}

template <int LP, int LA, int LB>
hipError_t launch_J(const JArgs &a, int grid, hipStream_t s) {
  using C = Cfg<LP, LA, LB>;
  constexpr int lds = JLayout<LP, LA, LB, C::TSJ, C::PCHJ>::BYTES_WG;
  auto kern = k_J<LP, LA, LB, C::TSJ, C::PCHJ>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::BLKJ), lds, s, a);
  return hipGetLastError();
}

template <int LP, int LA, int LB>
hipError_t launch_Jq(const JQArgs &a, int grid, hipStream_t s) {
  using C = Cfg<LP, LA, LB>;
  constexpr int lds = JLayout<LP, LA, LB, C::TSJ, C::PCHJ>::BYTES_WG;
  auto kern = k_Jq<LP, LA, LB, C::TSJ, C::PCHJ>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::BLKJ), lds, s, a);
  return hipGetLastError();
}

template <int LP, int LA, int LB>
hipError_t launch_gam(const GamArgs &a, int grid, hipStream_t s) {
  using C = Cfg<LP, LA, LB>;
  if constexpr (C::JREG) {
    auto kr = k_gam_r<LP, LA, LB>;
    int lds = a.nps * (a.pure ? 2 * LP + 1 : (LP + 1) * (LP + 2) / 2) * 8;
    if constexpr (GamSwap<LP>::ON) {
      if (a.nps > GamSwap<LP>::NPS) return hipErrorInvalidValue;
      lds += a.nps * ncart(LP) * 64 * 8;
    }
    hipLaunchKernelGGL(kr, dim3(grid), dim3(64), lds, s, a);
  } else {
    using E = GamE<LP, LA, LB>;
    auto kern = k_gam_e<LP, LA, LB>;
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    const int lds = (E::TEAM + a.nps * E::NCP) * 8;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(E::TS), lds, s, a);
  }
  return hipGetLastError();
}

template <int LP, int LQ>
hipError_t launch_metric(const MetArgs &a, int grid, hipStream_t s) {
  using C = Cfg<LP, LQ, 0>;
  constexpr int lds = C::LDS;
  auto kern = k_metric<LP, LQ, C::TS, C::PCH>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::BLK), lds, s, a);
  return hipGetLastError();
}

// metric classes (LP, LQ <= LP) of one LP
template <int LP, int LQ = 0>
void fill_metric(MetricInfo (&t)[7]) {
  using C = Cfg<LP, LQ, 0>;
  t[LQ].ppw = C::BLK / C::TS;
  t[LQ].fn = &launch_metric<LP, LQ>;
  if constexpr (LQ < LP) fill_metric<LP, LQ + 1>(t);
}

template <int LP, int LA, int LB>
hipError_t launch_grade(const GradArgs &a, int grid, int lds, hipStream_t s) {
  auto kern = k_grade<LP, LA, LB>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(ENG_TS), lds, s, a);
  return hipGetLastError();
}

template <int LP, int LA, int LB>
hipError_t launch_gradr(const GradArgs &a, int grid, int lds, hipStream_t s) {
  auto kern = k_gradr<LP, LA, LB>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <int LP, int LA, int LB>
GradInfo grad_info() {
  GradInfo g;
  if constexpr (GReg<LP, LA, LB>::OK) {
    g.tpb = 1;
    g.team = 0;
    g.ppw = 64;
    g.wpb = 1;
    g.gfn = &launch_gradr<LP, LA, LB>;
  } else {
    g.tpb = 1;
    g.team = GEng<LP, LA, LB>::TEAM;
    g.ppw = 1;
    g.wpb = ENG_TS / 64;
    g.min_aux = 8;
    g.gfn = &launch_grade<LP, LA, LB>;
  }
  return g;
}

template <int LP, int LA, int LB>
ClassInfo class_info() {
  using C = Cfg<LP, LA, LB>;
  ClassInfo c;
  c.ts = C::TS;
  c.tpw = C::BLK / C::TS;
  c.tpwj = C::BLKJ / C::TSJ;
  c.jreg = C::JREG ? 1 : 0;
  c.lds = C::STORE_LDS_V;
  c.store = &launch_store<LP, LA, LB>;
  // Cartesian-ket kernels of l <= 1 (the launches of the lower-degree terms
  // of l = 2, 3 run here); those of l >= 2 are registered by inst_cart_lp*
  if constexpr (LP <= 1) c.store_cart = &launch_store_cart<LP, LA, LB>;
  c.jfn = &launch_J<LP, LA, LB>;
  c.jq = &launch_Jq<LP, LA, LB>;
  c.gam = &launch_gam<LP, LA, LB>;
  return c;
}

constexpr int NLP = 7, NLA = 5;  // LP <= 6, la, lb <= 4
constexpr int NLG = 5;           // gradient: la, lb <= 4
// filled by inst_lp<LP>.hip
void register_metric_lp0(MetricInfo (&t)[7]);
void register_metric_lp1(MetricInfo (&t)[7]);
void register_metric_lp2(MetricInfo (&t)[7]);
void register_metric_lp3(MetricInfo (&t)[7]);
void register_metric_lp4(MetricInfo (&t)[7]);
void register_metric_lp5(MetricInfo (&t)[7]);
void register_metric_lp6(MetricInfo (&t)[7]);
void register_lp0(ClassInfo (&t)[NLA][NLA]);
void register_lp1(ClassInfo (&t)[NLA][NLA]);
void register_lp2(ClassInfo (&t)[NLA][NLA]);
void register_lp3(ClassInfo (&t)[NLA][NLA]);
void register_lp4(ClassInfo (&t)[NLA][NLA]);
void register_lp5(ClassInfo (&t)[NLA][NLA]);
void register_lp6(ClassInfo (&t)[NLA][NLA]);
void register_cart_lp2(ClassInfo (&t)[NLA][NLA]);
void register_cart_lp3(ClassInfo (&t)[NLA][NLA]);
void register_cart_lp4(ClassInfo (&t)[NLA][NLA]);
void register_cart_lp5(ClassInfo (&t)[NLA][NLA]);
void register_cart_lp6(ClassInfo (&t)[NLA][NLA]);
void register_grad_lp0(GradInfo (&t)[NLG][NLG]);
void register_grad_lp1(GradInfo (&t)[NLG][NLG]);
void register_grad_lp2(GradInfo (&t)[NLG][NLG]);
void register_grad_lp3(GradInfo (&t)[NLG][NLG]);
void register_grad_lp4(GradInfo (&t)[NLG][NLG]);
void register_grad_lp5(GradInfo (&t)[NLG][NLG]);
void register_grad_lp6(GradInfo (&t)[NLG][NLG]);

}  // namespace df3c

#define DF3C_REGISTER_LP(LPV, FN)                                   \
  namespace df3c {                                                  \
  void FN(ClassInfo (&t)[NLA][NLA]) {                               \
    t[0][0] = class_info<LPV, 0, 0>();                              \
    t[1][0] = class_info<LPV, 1, 0>();                              \
    t[1][1] = class_info<LPV, 1, 1>();                              \
    t[2][0] = class_info<LPV, 2, 0>();                              \
    t[2][1] = class_info<LPV, 2, 1>();                              \
    t[2][2] = class_info<LPV, 2, 2>();                              \
    t[3][0] = class_info<LPV, 3, 0>();                              \
    t[3][1] = class_info<LPV, 3, 1>();                              \
    t[3][2] = class_info<LPV, 3, 2>();                              \
    t[3][3] = class_info<LPV, 3, 3>();                              \
    t[4][0] = class_info<LPV, 4, 0>();                              \
    t[4][1] = class_info<LPV, 4, 1>();                              \
    t[4][2] = class_info<LPV, 4, 2>();                              \
    t[4][3] = class_info<LPV, 4, 3>();                              \
    t[4][4] = class_info<LPV, 4, 4>();                              \
  }                                                                 \
  }

#define DF3C_REGISTER_CART_LP(LPV, FN)                              \
  namespace df3c {                                                  \
  void FN(ClassInfo (&t)[NLA][NLA]) {                               \
    t[0][0].store_cart = &launch_store_cart<LPV, 0, 0>;             \
    t[1][0].store_cart = &launch_store_cart<LPV, 1, 0>;             \
    t[1][1].store_cart = &launch_store_cart<LPV, 1, 1>;             \
    t[2][0].store_cart = &launch_store_cart<LPV, 2, 0>;             \
    t[2][1].store_cart = &launch_store_cart<LPV, 2, 1>;             \
    t[2][2].store_cart = &launch_store_cart<LPV, 2, 2>;             \
    t[3][0].store_cart = &launch_store_cart<LPV, 3, 0>;             \
    t[3][1].store_cart = &launch_store_cart<LPV, 3, 1>;             \
    t[3][2].store_cart = &launch_store_cart<LPV, 3, 2>;             \
    t[3][3].store_cart = &launch_store_cart<LPV, 3, 3>;             \
    t[4][0].store_cart = &launch_store_cart<LPV, 4, 0>;             \
    t[4][1].store_cart = &launch_store_cart<LPV, 4, 1>;             \
    t[4][2].store_cart = &launch_store_cart<LPV, 4, 2>;             \
    t[4][3].store_cart = &launch_store_cart<LPV, 4, 3>;             \
    t[4][4].store_cart = &launch_store_cart<LPV, 4, 4>;             \
  }                                                                 \
  }

#define DF3C_REGISTER_GRAD_LP(LPV, FN)                              \
  namespace df3c {                                                  \
  void FN(GradInfo (&t)[NLG][NLG]) {                                \
    t[0][0] = grad_info<LPV, 0, 0>();                               \
    t[1][0] = grad_info<LPV, 1, 0>();                               \
    t[1][1] = grad_info<LPV, 1, 1>();                               \
    t[2][0] = grad_info<LPV, 2, 0>();                               \
    t[2][1] = grad_info<LPV, 2, 1>();                               \
    t[2][2] = grad_info<LPV, 2, 2>();                               \
    t[3][0] = grad_info<LPV, 3, 0>();                               \
    t[3][1] = grad_info<LPV, 3, 1>();                               \
    t[3][2] = grad_info<LPV, 3, 2>();                               \
    t[3][3] = grad_info<LPV, 3, 3>();                               \
    t[4][0] = grad_info<LPV, 4, 0>();                               \
    t[4][1] = grad_info<LPV, 4, 1>();                               \
    t[4][2] = grad_info<LPV, 4, 2>();                               \
    t[4][3] = grad_info<LPV, 4, 3>();                               \
    t[4][4] = grad_info<LPV, 4, 4>();                               \
  }                                                                 \
  }
