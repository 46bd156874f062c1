"""MI355X-native workload-balanced push-relabel max-flow (HIP, gfx950)."""
