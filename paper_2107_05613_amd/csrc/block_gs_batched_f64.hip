// Batched block Gauss-Seidel launches, FP64 vector blocks.
#define BGS_T double
#include "block_gs_batched.inl"
