"""Triple-DES (EDE) in ECB mode for the AMD MI355X (gfx950)."""
