// Kernels and launchers of the 6144-bit size class.
#define PMK_CLASS_BITS 6144
#include "kernels_class.inc"
