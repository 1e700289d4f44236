"""EBIC fitness evaluation on MI355X (gfx950)."""
