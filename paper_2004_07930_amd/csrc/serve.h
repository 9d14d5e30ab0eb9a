// Serving loop of libhz (continuous batching of solve requests), see serve.cpp.
#pragma once

#include "krylov.h"

namespace hz {
struct Serve;
}
