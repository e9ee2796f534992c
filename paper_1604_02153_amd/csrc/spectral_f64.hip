// FP64 instantiation of the pseudospectral operators.
#define SLNK_SPECTRAL_REAL double
#include "spectral_impl.hpp"

namespace slnk {
// the mixed-precision context's beta A: FP32 fields through the FP64 transform
template hipError_t spec_scale<double, float>(hipStream_t, const SpecGrid<double>&, int, const int*, SymbolParams, int,
                                              const float*, float*, const float*, cplx<double>*, cplx<double>*);
}  // namespace slnk
