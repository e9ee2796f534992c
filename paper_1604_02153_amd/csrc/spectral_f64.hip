// FP64 instantiation of the pseudospectral operators.
#define SLNK_SPECTRAL_REAL double
#include "spectral_impl.hpp"
