"""MI355X-native tensor-tomography hot path (forward projector, adjoint,
squared-loss + L2 gradient, L-BFGS) behind a C ABI, with a thin binding."""
