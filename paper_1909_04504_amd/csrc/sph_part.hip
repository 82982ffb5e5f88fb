// One (dimension, kernel, pair precision) of the library's launch sequences,
// chosen by SPH_PART_DIM, SPH_PART_KERNEL and SPH_PART_T at compile time
// (the build compiles this file once per combination, in parallel).
#include "sph_engine.hpp"

#if !defined(SPH_PART_DIM) || !defined(SPH_PART_KERNEL) || !defined(SPH_PART_T)
#error "SPH_PART_DIM, SPH_PART_KERNEL and SPH_PART_T must be defined"
#endif

template struct sph_host::Api<SPH_PART_DIM, SPH_PART_KERNEL, SPH_PART_T>;
