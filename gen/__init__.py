"""Seeded synthetic lattice inputs (gauge fields, sources); no method arithmetic."""
