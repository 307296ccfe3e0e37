// Kernels and launchers of the 2048-bit size class.
#define PMK_CLASS_BITS 2048
#include "kernels_class.inc"
