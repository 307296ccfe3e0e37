// Kernels and launchers of the 1024-bit size class.
#define PMK_CLASS_BITS 1024
#include "kernels_class.inc"
