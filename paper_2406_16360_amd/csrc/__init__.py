"""HIP sources and build script of libmirres."""
