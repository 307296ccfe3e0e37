// Kernels and launchers of the 8192-bit size class.
#define PMK_CLASS_BITS 8192
#include "kernels_class.inc"
