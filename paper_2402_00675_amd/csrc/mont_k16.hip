// Streaming, exponentiation and range kernels for 16-bit words.
#include "mont_dispatch.hpp"

MONT_INSTANTIATE_WIDTH(16)
