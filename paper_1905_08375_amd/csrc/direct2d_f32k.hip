// Instantiation unit of the specialised 2D direct kernel (f32k); see direct2d.inc.
#define NDL_D2_MODE 2
#include "direct2d.inc"
