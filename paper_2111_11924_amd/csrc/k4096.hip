// Kernels and launchers of the 4096-bit size class.
#define PMK_CLASS_BITS 4096
#include "kernels_class.inc"
