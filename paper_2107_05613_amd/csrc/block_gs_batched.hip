// Batched block Gauss-Seidel launchers: the launch shape for the active width.
#include "block_gs_batched.inl"
