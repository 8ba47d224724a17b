"""MI355X-native fast Slepian transform (HIP kernels behind a C ABI)."""
