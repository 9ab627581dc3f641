// Time-line kernels instantiated for double2 spinor storage (see k_line_impl.h).
#define TP_LINE_S double2
#define TP_LINE_SUFFIX f64
#include "k_line_impl.h"
