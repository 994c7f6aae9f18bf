"""Exact counting queries over a complete categorical database on MI355X."""
