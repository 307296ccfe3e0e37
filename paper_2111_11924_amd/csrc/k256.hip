// Kernels and launchers of the 256-bit size class.
#define PMK_CLASS_BITS 256
#include "kernels_class.inc"
