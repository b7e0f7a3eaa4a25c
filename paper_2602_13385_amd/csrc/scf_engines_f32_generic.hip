// Engine instances, float: generic instances (compiled nmax bound 20) for a set of degrees.
#include "scf_kernels.h"

namespace scf {

#define SCF_ENGINE(N, L)              \
  if (nmax <= N && lmax == L) { \
    static EngineImpl<float, N, L> e;   \
    return &e;                        \
  }

Engine* find_engine_f32_generic(int nmax, int lmax) {
  // any nmax <= 20 for these degrees
  SCF_ENGINE(20, 0)
  SCF_ENGINE(20, 1)
  SCF_ENGINE(20, 2)
  SCF_ENGINE(20, 3)
  SCF_ENGINE(20, 4)
  SCF_ENGINE(20, 5)
  SCF_ENGINE(20, 6)
  SCF_ENGINE(20, 7)
  SCF_ENGINE(20, 8)
  SCF_ENGINE(20, 9)
  SCF_ENGINE(20, 10)
  return nullptr;
}

#undef SCF_ENGINE

}  // namespace scf
