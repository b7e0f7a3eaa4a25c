// Engine instances, float: exact (nmax, lmax) instances for the shipped workloads.
#include "scf_kernels.h"

namespace scf {

#define SCF_ENGINE(N, L)              \
  if (nmax == N && lmax == L) { \
    static EngineImpl<float, N, L> e;   \
    return &e;                        \
  }

Engine* find_engine_f32_exact(int nmax, int lmax) {
  // exact-size instances for the shipped workloads
  SCF_ENGINE(6, 4)
  SCF_ENGINE(10, 5)
  SCF_ENGINE(10, 6)
  SCF_ENGINE(16, 10)
  return nullptr;
}

#undef SCF_ENGINE

}  // namespace scf
