"""MI355X spectral Ewald (periodic Stokeslet) library."""
