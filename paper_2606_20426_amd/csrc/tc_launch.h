// Host-side launch interface of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "tc_device.h"

namespace tc {

enum class KernelId : int {
  setup_tets,
  setup_mass,
  setup_area,
  predict,
  project,
  element,
  barrier,
  asm_diag,
  asm_off,
  newton_begin,
  cg_spmv,
  cg_update,
  newton_dir,
  filter,
  env_dir,
  energy,
  env_ls,
  update,
  env_update,
  sigma,
  traction,
  contact,
  env_extract,
  commit,
  pairs,
  pair_push,
  pair_apply,
  count
};

inline const char* kernel_name(KernelId k) {
  static const char* names[] = {"setup_tets", "setup_mass", "setup_area", "predict",   "project",
                                "element",    "barrier",    "asm_diag",   "asm_off",   "newton_begin",
                                "cg_spmv",    "cg_update",  "newton_dir", "filter",    "env_dir",
                                "energy",     "env_ls",     "update",     "env_update", "sigma",     "traction",
                                "contact",    "env_extract", "commit",     "pairs",     "pair_push",
                                "pair_apply"};
  return names[static_cast<int>(k)];
}

struct LaunchArgs {
  const Tile* tiles = nullptr;
  int ntiles = 0;
  int block = 256;
  const EnvDesc* envs = nullptr;
  int n_env = 0;
  int parity = 0;
  int mode = 0;
  int lpr = 0;             // SpMV lanes per row (16, 32; 0 = one thread per row)
  double* out = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr;    // timing: recorded at the dispatch's start and end
  hipEvent_t ev1 = nullptr;
  // timing of the CG kernels from inside: (start, end) GPU wall clock of
  // every block, 2 x u64 per block (zero-initialised)
  unsigned long long* clock = nullptr;
};

// Kernels that time themselves with the GPU wall clock when given a slot.
inline bool self_timed(KernelId k) {
  return k == KernelId::cg_spmv || k == KernelId::cg_update;
}

// Launch errors surface through hipGetLastError.
hipError_t launch_kernel(KernelId id, bool fp64, const LaunchArgs& a);

}  // namespace tc
