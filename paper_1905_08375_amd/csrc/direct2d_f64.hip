// Instantiation unit of the specialised 2D direct kernel (f64); see direct2d.inc.
#define NDL_D2_MODE 0
#include "direct2d.inc"
