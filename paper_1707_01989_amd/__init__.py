"""Cooperative kernels for blocking graph traversal on MI355X (gfx950)."""
