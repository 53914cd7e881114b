"""MI355X-native fused-pack GEMM (packing fused with the first computational pass)."""
