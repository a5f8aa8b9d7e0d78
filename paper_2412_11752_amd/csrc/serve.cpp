// Serving loop (continuous batching).  Filled in below.
#include "drk_internal.hpp"
