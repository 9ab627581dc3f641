// Time-line kernels instantiated for __half2 spinor storage (see k_line_impl.h).
#define TP_LINE_S __half2
#define TP_LINE_SUFFIX f16
#include "k_line_impl.h"
