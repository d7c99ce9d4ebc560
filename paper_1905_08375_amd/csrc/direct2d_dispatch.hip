// Instantiation unit of the specialised 2D direct kernel (dispatch); see direct2d.inc.
#define NDL_D2_MODE -1
#include "direct2d.inc"
