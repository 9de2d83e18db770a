"""MI355X-native FReSCo loss + gradient engine (HIP kernels behind a C ABI)."""
