// Kernels and launchers of the 128-bit size class.
#define PMK_CLASS_BITS 128
#include "kernels_class.inc"
