// Streaming, exponentiation and range kernels for 32-bit words.
#include "mont_dispatch.hpp"

MONT_INSTANTIATE_WIDTH(32)
