// Temporally blocked leapfrog (several substeps per launch): not built yet.
#pragma once

#include "common.hpp"

namespace hgs {

constexpr bool kTBlockAvailable = false;

template <typename S>
void launch_tblock(const S*, const S*, const S*, S*, S*, const Layout&, const StepCoef&, int, hipStream_t) {}

}  // namespace hgs
