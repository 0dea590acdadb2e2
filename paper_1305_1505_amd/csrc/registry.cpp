// Map (N, precision) to the launcher table instantiated for it.
#include "ops.hpp"
#include "sizes.hpp"

namespace pin {

#define PIN_DECL(n) \
  const SizeOps* ops_0_##n(); \
  const SizeOps* ops_1_##n();
PIN_FOR_EACH_SIZE(PIN_DECL)
#undef PIN_DECL

const SizeOps* find_ops(int n, bool fp64) {
  switch (n) {
#define PIN_CASE(v) \
  case v: return fp64 ? ops_1_##v() : ops_0_##v();
    PIN_FOR_EACH_SIZE(PIN_CASE)
#undef PIN_CASE
    default: return nullptr;
  }
}

}  // namespace pin
