"""HIP sources of libgsis and their build script."""
