// Time-line kernels instantiated for float2 spinor storage (see k_line_impl.h).
#define TP_LINE_S float2
#define TP_LINE_SUFFIX f32
#include "k_line_impl.h"
