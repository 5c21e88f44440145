"""Exact cone-beam system matrix (arXiv 2511.12235) on MI355X."""
