// Common includes of every kernel translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "devmath.hpp"
#include "plan.hpp"
