// Kernels and launchers of the 512-bit size class.
#define PMK_CLASS_BITS 512
#include "kernels_class.inc"
