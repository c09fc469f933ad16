// Persistent ragged-batch kernels (filled in below).
#include "lap_kernels.hpp"
namespace lap {}
