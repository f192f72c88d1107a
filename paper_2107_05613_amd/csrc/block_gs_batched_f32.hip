// Batched block Gauss-Seidel launches, FP32 vector blocks.
#define BGS_T float
#include "block_gs_batched.inl"
