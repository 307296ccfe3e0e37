// Kernels and launchers of the 3072-bit size class.
#define PMK_CLASS_BITS 3072
#include "kernels_class.inc"
