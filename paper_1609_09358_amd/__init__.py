"""Hybrid BP -> CA-SCL polar decoder for MI355X (gfx950)."""
