"""MI355X-native flood GaBP solver (arXiv 1904.04093) behind a C-ABI HIP library."""
