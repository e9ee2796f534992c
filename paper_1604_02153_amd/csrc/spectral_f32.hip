// FP32 instantiation of the pseudospectral operators.
#define SLNK_SPECTRAL_REAL float
#include "spectral_impl.hpp"
