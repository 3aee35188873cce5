// elgamal.hpp -- internal: the per-device fixed-base table of the generator.
#pragma once
#include <stdint.h>

#include "../../include/pcmm.h"

namespace pcmm {

// 4-bit window table of G (960 affine points, Montgomery form, structure of
// arrays with ld 960), built on the current device on first use.
pcmm_status generator_table(const uint32_t **out);

}  // namespace pcmm
